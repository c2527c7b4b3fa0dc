// phsp_serve.hip -- continuous-batching request server.
//
// Host scheduler over the multi-channel kernel: a FIFO queue, an
// HBM arena with a first-fit free list (the budget), a ring of tick slots
// (pinned staging + device tables), and one in-order stream on which ticks run
// back to back.  Every request is cut into tiles of kBlock events; a tick takes
// tiles from the active requests, oldest first, and merges the partial sums of
// the requests whose last tile it holds.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hydra_phsp.h"
#include "hydra_phsp_serve.h"
#include "phsp_api_internal.hpp"
#include "phsp_batch.hpp"

namespace hphsp {
namespace {

constexpr int kServeEpt = 1; // a tile is kBlock events, one per thread
static_assert(kServeEpt == 1, "the mixed-N kernels of a tick are built with one event per thread");
constexpr uint64_t kAlign = 256;
constexpr int kTickSlots = 4;

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device allocation.
class Arena {
  public:
    bool init(uint64_t bytes) {
        size_ = bytes;
        if (hipMalloc(&base_, bytes) != hipSuccess) {
            base_ = nullptr;
            return false;
        }
        free_[0] = bytes;
        return true;
    }
    void destroy() {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
    }
    // Returns false when no free range is large enough.
    bool alloc(uint64_t bytes, uint64_t* off) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes;
                const uint64_t roff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[roff] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    char* ptr(uint64_t off) const { return base_ + off; }
    uint64_t size() const { return size_; }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }

  private:
    char* base_ = nullptr;
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;
};

uint64_t round_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Request {
    hydra_phsp_request r;
    Channel ch;
    uint64_t ntiles = 0, next_tile = 0;
    uint64_t off = 0, bytes = 0;
    double* out = nullptr;
    double* weights = nullptr;
    Moments* parts = nullptr;
    bool admitted = false, done = false;
    hydra_phsp_result res;
};

// Per-request device footprint: outputs (generate only) + one partial per tile.
uint64_t request_bytes(const hydra_phsp_request& r, uint64_t ntiles) {
    uint64_t b = round_up(sizeof(Moments) * ntiles);
    if (!r.integrate_only) {
        b += round_up(sizeof(double) * 4 * (uint64_t)r.n_daughters * r.nevents);
        b += round_up(sizeof(double) * r.nevents);
    }
    return b;
}

template <typename T>
struct Staged { // pinned host + device buffer pair, grown on demand
    T* host = nullptr;
    T* dev = nullptr;
    size_t cap = 0;
    int ensure(size_t n) {
        if (n <= cap) return HYDRA_PHSP_OK;
        size_t c = std::max<size_t>(cap ? cap : 64, 64);
        while (c < n) c *= 2;
        free_all();
        if (hipHostMalloc(&host, sizeof(T) * c, hipHostMallocDefault) != hipSuccess) {
            host = nullptr;
            return fail(HYDRA_PHSP_ENOMEM, "server staging allocation failed");
        }
        if (hipMalloc(&dev, sizeof(T) * c) != hipSuccess) {
            dev = nullptr;
            return fail(HYDRA_PHSP_ENOMEM, "server table allocation failed");
        }
        cap = c;
        return HYDRA_PHSP_OK;
    }
    void free_all() {
        if (host) (void)hipHostFree(host);
        if (dev) (void)hipFree(dev);
        host = nullptr;
        dev = nullptr;
        cap = 0;
    }
};

struct TickSlot {
    Staged<DevChannel> chans;   // channels whose tiles this tick processes
    Staged<TileRef> tiles;
    Staged<DevChannel> fin;     // requests finishing in this tick (merge records)
    Staged<GroupRef> groups;
    Staged<double> stats;       // 4 per finishing request (device -> pinned host)
    Moments* mid = nullptr;
    size_t mid_cap = 0;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> finishing;
};

} // namespace
} // namespace hphsp

using namespace hphsp;

struct hydra_phsp_server {
    int device = 0;
    int cus = 256;
    uint64_t max_tiles_per_tick = 0;
    int max_active = 1024;
    Arena arena;
    hipStream_t stream = nullptr;
    const double2* trig = nullptr;
    TickSlot slots[kTickSlots];
    int next_slot = 0;
    std::deque<int> busy_order; // slots in launch order
    std::mutex mu;              // guards queue, reqs, next_id (submit may run on any thread)
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, Request> reqs;
    uint64_t next_id = 1;
    std::vector<uint64_t> active; // admitted with tiles left, in admission order
    std::vector<uint64_t> completed;
    uint64_t ticks = 0, finished = 0;
    uint64_t budget_stalls = 0, active_stalls = 0;
    double queue_wait_max = 0.0, queue_wait_sum = 0.0;
};

namespace hphsp {
namespace {

int validate_request(const hydra_phsp_request& r, Channel* ch) {
    int st = make_channel(r.parent_mass, r.masses, r.n_daughters, ch);
    if (st != HYDRA_PHSP_OK) return st;
    if (r.nevents < 1) return fail(HYDRA_PHSP_EINVAL, "request needs nevents >= 1");
    if (r.nevents > (1ull << 40)) return fail(HYDRA_PHSP_EINVAL, "request too large");
    return HYDRA_PHSP_OK;
}

int retire(hydra_phsp_server* s) {
    while (!s->busy_order.empty()) {
        TickSlot& t = s->slots[s->busy_order.front()];
        const hipError_t q = hipEventQuery(t.done);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess) return fail_hip(q, "tick completion");
        const double now = now_s();
        std::lock_guard<std::mutex> lock(s->mu);
        for (size_t k = 0; k < t.finishing.size(); ++k) {
            auto it = s->reqs.find(t.finishing[k]);
            if (it == s->reqs.end()) continue;
            Request& r = it->second;
            r.res.mean = t.stats.host[4 * k + 1];
            r.res.sigma = t.stats.host[4 * k + 3];
            r.res.status = HYDRA_PHSP_OK;
            r.res.done_s = now;
            r.done = true;
            const double waited = r.res.admit_s - r.res.submit_s;
            s->queue_wait_sum += waited;
            s->queue_wait_max = std::max(s->queue_wait_max, waited);
            s->completed.push_back(t.finishing[k]);
            ++s->finished;
        }
        t.finishing.clear();
        t.busy = false;
        s->busy_order.pop_front();
    }
    return HYDRA_PHSP_OK;
}

void admit(hydra_phsp_server* s) {
    std::lock_guard<std::mutex> lock(s->mu);
    const double now = now_s();
    while (!s->queue.empty()) {
        if ((int)s->active.size() >= s->max_active) {
            ++s->active_stalls;
            break;
        }
        Request& r = s->reqs[s->queue.front()];
        if (!s->arena.alloc(r.bytes, &r.off)) { // FIFO: wait for memory
            ++s->budget_stalls;
            break;
        }
        char* p = s->arena.ptr(r.off);
        r.parts = reinterpret_cast<Moments*>(p);
        p += round_up(sizeof(Moments) * r.ntiles);
        if (!r.r.integrate_only) {
            r.out = reinterpret_cast<double*>(p);
            p += round_up(sizeof(double) * 4 * (uint64_t)r.r.n_daughters * r.r.nevents);
            r.weights = reinterpret_cast<double*>(p);
        }
        r.admitted = true;
        r.res.admit_s = now;
        r.res.p4_dev = r.out;
        r.res.weights_dev = r.weights;
        s->active.push_back(s->queue.front());
        s->queue.pop_front();
    }
}

DevChannel dev_channel(const Request& r) {
    DevChannel d;
    std::memset(&d, 0, sizeof(d));
    d.a.ch = r.ch;
    d.a.nevents = r.r.nevents;
    d.a.event_offset = 0;
    d.a.k0 = (uint32_t)(r.r.seed & 0xFFFFFFFFu);
    d.a.k1 = (uint32_t)(r.r.seed >> 32);
    d.a.sid = r.r.stream_id;
    d.a.out = r.out;
    d.a.ld = r.r.nevents;
    d.a.weights = r.weights;
    d.a.inv_M = 1.0 / r.ch.M;
    d.a.partials = r.parts;
    d.n = r.r.n_daughters;
    d.mode = r.r.integrate_only ? kIntegrate : kFp64;
    d.ntiles = r.ntiles;
    d.ngroups = stage1_groups(r.ntiles);
    return d;
}

int launch_tick(hydra_phsp_server* s) {
    if (s->active.empty()) return HYDRA_PHSP_OK;
    TickSlot& t = s->slots[s->next_slot];
    if (t.busy) return HYDRA_PHSP_OK; // all slots in flight: wait for the GPU
    std::vector<DevChannel> chans;
    std::vector<TileRef> tiles;
    std::vector<DevChannel> fin;
    std::vector<GroupRef> groups;
    std::vector<uint64_t> finishing;
    // The tick is planned without touching the requests; their progress (next
    // tile, leaving the active list) is committed only once the tick is on the
    // stream, so a failure below leaves every request as it was.
    std::vector<std::pair<uint64_t, uint64_t>> progress; // (request, its next tile after this tick)
    std::vector<uint64_t> still;
    int nmax = 2;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        for (uint64_t id : s->active) {
            Request& r = s->reqs[id];
            if (tiles.size() < s->max_tiles_per_tick && r.next_tile < r.ntiles) {
                const uint32_t ci = (uint32_t)chans.size();
                chans.push_back(dev_channel(r));
                nmax = std::max(nmax, r.r.n_daughters);
                uint64_t next = r.next_tile;
                while (next < r.ntiles && tiles.size() < s->max_tiles_per_tick) tiles.push_back(TileRef{ci, 0u, next++});
                progress.emplace_back(id, next);
                if (next == r.ntiles) {
                    DevChannel f = dev_channel(r);
                    f.first_group = groups.size();
                    for (uint64_t g = 0; g < f.ngroups; ++g) groups.push_back(GroupRef{(uint32_t)fin.size(), (uint32_t)g});
                    fin.push_back(f);
                    finishing.push_back(id);
                    continue; // leaves the active list
                }
            }
            still.push_back(id);
        }
    }
    if (tiles.empty()) return HYDRA_PHSP_OK;
    int st = t.chans.ensure(chans.size());
    if (st == HYDRA_PHSP_OK) st = t.tiles.ensure(tiles.size());
    if (st == HYDRA_PHSP_OK) st = t.fin.ensure(std::max<size_t>(fin.size(), 1));
    if (st == HYDRA_PHSP_OK) st = t.groups.ensure(std::max<size_t>(groups.size(), 1));
    if (st == HYDRA_PHSP_OK) st = t.stats.ensure(std::max<size_t>(4 * fin.size(), 4));
    if (st == HYDRA_PHSP_OK && groups.size() > t.mid_cap) {
        if (t.mid) (void)hipFree(t.mid);
        size_t c = std::max<size_t>(t.mid_cap ? t.mid_cap : 64, 64);
        while (c < groups.size()) c *= 2;
        if (hipMalloc(&t.mid, sizeof(Moments) * c) != hipSuccess) {
            t.mid = nullptr;
            t.mid_cap = 0;
            st = fail(HYDRA_PHSP_ENOMEM, "server merge buffer allocation failed");
        } else {
            t.mid_cap = c;
        }
    }
    if (st != HYDRA_PHSP_OK) return st;
    for (size_t k = 0; k < fin.size(); ++k) fin[k].stats = t.stats.dev + 4 * k;
    std::memcpy(t.chans.host, chans.data(), sizeof(DevChannel) * chans.size());
    std::memcpy(t.tiles.host, tiles.data(), sizeof(TileRef) * tiles.size());
    if (!fin.empty()) {
        std::memcpy(t.fin.host, fin.data(), sizeof(DevChannel) * fin.size());
        std::memcpy(t.groups.host, groups.data(), sizeof(GroupRef) * groups.size());
    }
    hipStream_t q = s->stream;
    hipError_t e = hipMemcpyAsync(t.chans.dev, t.chans.host, sizeof(DevChannel) * chans.size(),
                                  hipMemcpyHostToDevice, q);
    if (e == hipSuccess)
        e = hipMemcpyAsync(t.tiles.dev, t.tiles.host, sizeof(TileRef) * tiles.size(), hipMemcpyHostToDevice, q);
    if (e == hipSuccess && !fin.empty()) {
        e = hipMemcpyAsync(t.fin.dev, t.fin.host, sizeof(DevChannel) * fin.size(), hipMemcpyHostToDevice, q);
        if (e == hipSuccess)
            e = hipMemcpyAsync(t.groups.dev, t.groups.host, sizeof(GroupRef) * groups.size(),
                               hipMemcpyHostToDevice, q);
    }
    if (e != hipSuccess) return fail_hip(e, "server table upload");
    // One block per tile: blocks are dispatched in tile order, so each request's
    // output columns are written front to back.
    BatchLaunch b{t.chans.dev, t.tiles.dev, (uint64_t)tiles.size(),
                  std::min<uint64_t>((uint64_t)tiles.size(), kMaxGridBlocks), s->trig, nullptr};
    e = launch_mixed_tiles(nmax, 1, b, q);
    if (e != hipSuccess) return fail_hip(e, "server tick launch");
    if (!fin.empty()) {
        e = launch_batch_merges(t.fin.dev, t.groups.dev, groups.size(), t.mid, fin.size(), q);
        if (e == hipSuccess)
            e = hipMemcpyAsync(t.stats.host, t.stats.dev, sizeof(double) * 4 * fin.size(), hipMemcpyDeviceToHost, q);
        if (e != hipSuccess) return fail_hip(e, "server merge launch");
    }
    e = hipEventRecord(t.done, q);
    if (e != hipSuccess) return fail_hip(e, "hipEventRecord");
    {
        std::lock_guard<std::mutex> lock(s->mu);
        for (const auto& pr : progress) s->reqs[pr.first].next_tile = pr.second;
        s->active.swap(still);
        ++s->ticks;
    }
    t.finishing.swap(finishing);
    t.busy = true;
    s->busy_order.push_back(s->next_slot);
    s->next_slot = (s->next_slot + 1) % kTickSlots;
    return HYDRA_PHSP_OK;
}

int pending(hydra_phsp_server* s) {
    std::lock_guard<std::mutex> lock(s->mu);
    size_t inflight = 0;
    for (int i = 0; i < kTickSlots; ++i) inflight += s->slots[i].finishing.size();
    return (int)(s->queue.size() + s->active.size() + inflight);
}

void free_server(hydra_phsp_server* s) {
    for (int i = 0; i < kTickSlots; ++i) {
        TickSlot& t = s->slots[i];
        t.chans.free_all();
        t.tiles.free_all();
        t.fin.free_all();
        t.groups.free_all();
        t.stats.free_all();
        if (t.mid) (void)hipFree(t.mid);
        if (t.done) (void)hipEventDestroy(t.done);
    }
    s->arena.destroy();
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

} // namespace
} // namespace hphsp

extern "C" {

int hydra_phsp_server_create(uint64_t hbm_budget_bytes, uint64_t max_events_per_tick, int max_active,
                             hydra_phsp_server** server_out) {
    if (server_out == nullptr) return fail(HYDRA_PHSP_EINVAL, "server_out is NULL");
    if (hbm_budget_bytes < (1ull << 20)) return fail(HYDRA_PHSP_EINVAL, "budget must be at least 1 MiB");
    if (max_active < 0) return fail(HYDRA_PHSP_EINVAL, "max_active must be >= 0");
    hydra_phsp_server* s = new hydra_phsp_server();
    if (max_events_per_tick == 0) max_events_per_tick = 1ull << 22;
    s->max_tiles_per_tick = std::max<uint64_t>(1, max_events_per_tick / (uint64_t)kBlock);
    if (max_active > 0) s->max_active = max_active;
    hipError_t e = hipGetDevice(&s->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device);
    if (e != hipSuccess) {
        delete s;
        return fail_hip(e, "hipGetDevice");
    }
    int tst = trig_table(&s->trig);
    if (tst != HYDRA_PHSP_OK) {
        delete s;
        return tst;
    }
    if (!s->arena.init(hbm_budget_bytes)) {
        delete s;
        return fail(HYDRA_PHSP_ENOMEM, "server arena allocation failed");
    }
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    for (int i = 0; e == hipSuccess && i < kTickSlots; ++i)
        e = hipEventCreateWithFlags(&s->slots[i].done, hipEventDisableTiming);
    if (e != hipSuccess) {
        free_server(s);
        return fail_hip(e, "server stream/event creation");
    }
    *server_out = s;
    return HYDRA_PHSP_OK;
}

int hydra_phsp_server_submit(hydra_phsp_server* s, const hydra_phsp_request* req, uint64_t* id_out) {
    if (s == nullptr || req == nullptr || id_out == nullptr) return fail(HYDRA_PHSP_EINVAL, "NULL argument");
    Request r;
    r.r = *req;
    int st = validate_request(*req, &r.ch);
    if (st != HYDRA_PHSP_OK) return st;
    r.ntiles = (req->nevents + kBlock - 1) / kBlock;
    r.bytes = request_bytes(*req, r.ntiles);
    if (r.bytes > s->arena.size()) return fail(HYDRA_PHSP_ENOMEM, "request larger than the server's HBM budget");
    std::memset(&r.res, 0, sizeof(r.res));
    r.res.status = HYDRA_PHSP_EAGAIN;
    r.res.n_daughters = req->n_daughters;
    r.res.nevents = req->nevents;
    r.res.submit_s = now_s();
    std::lock_guard<std::mutex> lock(s->mu);
    const uint64_t id = s->next_id++;
    s->reqs.emplace(id, r);
    s->queue.push_back(id);
    *id_out = id;
    return HYDRA_PHSP_OK;
}

int hydra_phsp_server_step(hydra_phsp_server* s) {
    MarkerRange marker("hydra_phsp_server_step");
    if (s == nullptr) return fail(HYDRA_PHSP_EINVAL, "server is NULL");
    int st = retire(s);
    if (st != HYDRA_PHSP_OK) return st;
    admit(s);
    st = launch_tick(s);
    if (st != HYDRA_PHSP_OK) return st;
    return pending(s);
}

int hydra_phsp_server_completed(hydra_phsp_server* s, uint64_t* ids_out, int max) {
    if (s == nullptr || (ids_out == nullptr && max > 0)) return fail(HYDRA_PHSP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    const int n = std::min<int>(max, (int)s->completed.size());
    for (int i = 0; i < n; ++i) ids_out[i] = s->completed[i];
    s->completed.erase(s->completed.begin(), s->completed.begin() + n);
    return n;
}

int hydra_phsp_server_poll(hydra_phsp_server* s, uint64_t id, hydra_phsp_result* res) {
    if (s == nullptr || res == nullptr) return fail(HYDRA_PHSP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(HYDRA_PHSP_ENOTFOUND, "unknown request id");
    *res = it->second.res;
    return it->second.done ? HYDRA_PHSP_OK : HYDRA_PHSP_EAGAIN;
}

int hydra_phsp_server_release(hydra_phsp_server* s, uint64_t id) {
    if (s == nullptr) return fail(HYDRA_PHSP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(HYDRA_PHSP_ENOTFOUND, "unknown request id");
    if (!it->second.done) return fail(HYDRA_PHSP_EAGAIN, "request has not finished");
    s->arena.release(it->second.off, it->second.bytes);
    s->reqs.erase(it);
    return HYDRA_PHSP_OK;
}

int hydra_phsp_server_drain(hydra_phsp_server* s) {
    if (s == nullptr) return fail(HYDRA_PHSP_EINVAL, "server is NULL");
    for (;;) {
        const int p = hydra_phsp_server_step(s);
        if (p < 0) return p;
        if (p == 0) return HYDRA_PHSP_OK;
        bool queued_only;
        {
            std::lock_guard<std::mutex> lock(s->mu);
            queued_only = s->active.empty() && s->busy_order.empty() && !s->queue.empty();
        }
        // Queued requests that cannot be admitted while nothing runs never will.
        if (queued_only) {
            admit(s);
            std::lock_guard<std::mutex> lock(s->mu);
            if (s->active.empty()) return fail(HYDRA_PHSP_ENOMEM, "queued requests exceed the free budget");
        }
        if (!s->busy_order.empty()) (void)hipEventSynchronize(s->slots[s->busy_order.front()].done);
    }
}

int hydra_phsp_server_replay(hydra_phsp_server* s, const hydra_phsp_request* reqs, const double* arrival_s, int n,
                             double* latency_s_out, double* wall_s_out, uint64_t* peak_bytes_out) {
    MarkerRange marker("hydra_phsp_server_replay");
    if (s == nullptr || (n > 0 && (reqs == nullptr || arrival_s == nullptr || latency_s_out == nullptr)))
        return fail(HYDRA_PHSP_EINVAL, "NULL argument");
    std::unordered_map<uint64_t, int> index;
    const double t0 = now_s();
    int next = 0, done = 0;
    std::vector<uint64_t> ids(256);
    while (done < n) {
        const double now = now_s() - t0;
        while (next < n && arrival_s[next] <= now) {
            uint64_t id = 0;
            if (hydra_phsp_server_submit(s, &reqs[next], &id) == HYDRA_PHSP_OK) {
                index[id] = next;
            } else {
                latency_s_out[next] = -1.0;
                ++done;
            }
            ++next;
        }
        const int p = hydra_phsp_server_step(s);
        if (p < 0) return p;
        int got;
        while ((got = hydra_phsp_server_completed(s, ids.data(), (int)ids.size())) > 0) {
            for (int k = 0; k < got; ++k) {
                hydra_phsp_result r;
                (void)hydra_phsp_server_poll(s, ids[k], &r);
                const int i = index[ids[k]];
                latency_s_out[i] = r.done_s - (t0 + arrival_s[i]);
                (void)hydra_phsp_server_release(s, ids[k]);
                index.erase(ids[k]);
                ++done;
            }
        }
        if (p == 0 && next < n) {
            const double wait = arrival_s[next] - (now_s() - t0);
            if (wait > 50e-6) std::this_thread::sleep_for(std::chrono::microseconds((long)(wait * 0.5e6)));
        }
    }
    if (wall_s_out) *wall_s_out = now_s() - t0;
    if (peak_bytes_out) *peak_bytes_out = s->arena.peak();
    return HYDRA_PHSP_OK;
}

int hydra_phsp_server_stats(const hydra_phsp_server* s, uint64_t* bytes_in_use, uint64_t* peak_bytes,
                            uint64_t* ticks, uint64_t* finished) {
    if (s == nullptr) return fail(HYDRA_PHSP_EINVAL, "server is NULL");
    if (bytes_in_use) *bytes_in_use = s->arena.used();
    if (peak_bytes) *peak_bytes = s->arena.peak();
    if (ticks) *ticks = s->ticks;
    if (finished) *finished = s->finished;
    return HYDRA_PHSP_OK;
}

int hydra_phsp_server_counters_get(const hydra_phsp_server* s, hydra_phsp_server_counters* out) {
    if (s == nullptr || out == nullptr) return fail(HYDRA_PHSP_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lock(const_cast<hydra_phsp_server*>(s)->mu);
    out->bytes_in_use = s->arena.used();
    out->peak_bytes = s->arena.peak();
    out->ticks = s->ticks;
    out->finished = s->finished;
    out->budget_stalls = s->budget_stalls;
    out->active_stalls = s->active_stalls;
    out->queue_wait_max_s = s->queue_wait_max;
    out->queue_wait_sum_s = s->queue_wait_sum;
    return HYDRA_PHSP_OK;
}

int hydra_phsp_server_destroy(hydra_phsp_server* s) {
    if (s == nullptr) return fail(HYDRA_PHSP_EINVAL, "server is NULL");
    int st = HYDRA_PHSP_OK;
    if (s->stream) {
        hipError_t e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) st = fail_hip(e, "hipStreamSynchronize");
    }
    free_server(s);
    return st;
}

} // extern "C"

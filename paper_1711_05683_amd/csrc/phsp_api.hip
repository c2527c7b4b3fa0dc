// phsp_api.hip -- C ABI of the single-channel path: argument validation,
// per-channel constants, workspace management and launches.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hydra_phsp.h"
#include "phsp_api_internal.hpp"
#include "phsp_ept.hpp"
#include "phsp_finalize.hpp"
#include "phsp_kernels.hpp"

namespace hphsp {

// ---------------------------------------------------------------- errors ----

static thread_local std::string t_last_error;

int fail(int status, const std::string& msg) {
    t_last_error = msg;
    return status;
}

int fail_hip(hipError_t e, const char* what) {
    t_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return HYDRA_PHSP_EDEVICE;
}

// ------------------------------------------------------------- validation ----

int make_channel(double M, const double* masses, int n, Channel* out) {
    if (n < 2 || n > kNMax) return fail(HYDRA_PHSP_EINVAL, "n_daughters must be in [2, 10]");
    if (masses == nullptr) return fail(HYDRA_PHSP_EINVAL, "masses_host is NULL");
    if (!std::isfinite(M) || !(M > 0.0)) return fail(HYDRA_PHSP_EINVAL, "parent mass must be finite and > 0");
    Channel c;
    std::memset(&c, 0, sizeof(c));
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!std::isfinite(masses[i]) || !(masses[i] >= 0.0))
            return fail(HYDRA_PHSP_EINVAL, "daughter masses must be finite and >= 0");
        s += masses[i];
        c.m[i] = masses[i];
        c.S[i] = s;
    }
    const double T = M - s;
    if (!(T > 0.0)) return fail(HYDRA_PHSP_EKINEMATICS, "parent mass must exceed the sum of daughter masses");
    // C = pi^{N-1} (2T)^{N-2} / (M (N-2)!): the volume of the sorted-uniform
    // simplex and the Jacobian d(sigma^2) -> 2 sigma T dR of each inner level.
    double C = 1.0 / M;
    for (int i = 0; i < n - 1; ++i) C *= 3.141592653589793;
    for (int i = 0; i < n - 2; ++i) C *= 2.0 * T;
    for (int i = 2; i <= n - 2; ++i) C /= (double)i;
    c.M = M;
    c.T = T;
    c.C = C;
    c.half_inv_M = 0.5 / M;
    *out = c;
    return HYDRA_PHSP_OK;
}

int make_frame(double M, const double* p4, Frame* f) {
    const double E = p4[0], px = p4[1], py = p4[2], pz = p4[3];
    if (!std::isfinite(E) || !std::isfinite(px) || !std::isfinite(py) || !std::isfinite(pz) || !(E > 0.0))
        return fail(HYDRA_PHSP_EINVAL, "parent four-vector must be finite with E > 0");
    const double m2 = E * E - (px * px + py * py + pz * pz);
    if (std::fabs(m2 - M * M) > 1e-9 * E * E)
        return fail(HYDRA_PHSP_EINVAL, "parent four-vector's invariant mass differs from parent_mass");
    f->eta[0] = px / M;
    f->eta[1] = py / M;
    f->eta[2] = pz / M;
    f->gamma = E / M;
    f->inv_gp1 = M / (E + M);
    return HYDRA_PHSP_OK;
}

// --------------------------------------------------------------- workspace ----

struct Workspace {
    Moments* mid = nullptr;       // kMaxGroups stage-1 results
    Moments* partials = nullptr;
    uint64_t capacity = 0;
    double* stats_host = nullptr; // pinned, HYDRA_PHSP_STATS doubles
    double* stats_dev = nullptr;  // HYDRA_PHSP_STATS doubles
};

static std::mutex g_ws_mutex;
static std::map<std::pair<int, hipStream_t>, Workspace> g_ws;

int workspace_for(hipStream_t stream, uint64_t partials, Workspace** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    Workspace& w = g_ws[std::make_pair(dev, stream)];
    if (w.stats_dev == nullptr) {
        e = hipMalloc(&w.stats_dev, sizeof(double) * HYDRA_PHSP_STATS);
        if (e != hipSuccess) return fail(HYDRA_PHSP_ENOMEM, "workspace allocation failed");
        e = hipMalloc(&w.mid, sizeof(Moments) * kMaxGroups);
        if (e != hipSuccess) return fail(HYDRA_PHSP_ENOMEM, "workspace allocation failed");
        e = hipHostMalloc(&w.stats_host, sizeof(double) * HYDRA_PHSP_STATS, hipHostMallocDefault);
        if (e != hipSuccess) return fail(HYDRA_PHSP_ENOMEM, "pinned workspace allocation failed");
    }
    if (partials > w.capacity) {
        uint64_t cap = w.capacity ? w.capacity : 4096;
        while (cap < partials) cap *= 2;
        if (w.partials != nullptr) {
            // hipFree waits for the device, so no queued kernel still reads it.
            e = hipFree(w.partials);
            if (e != hipSuccess) return fail_hip(e, "hipFree");
            w.partials = nullptr;
            w.capacity = 0;
        }
        e = hipMalloc(&w.partials, sizeof(Moments) * cap);
        if (e != hipSuccess) return fail(HYDRA_PHSP_ENOMEM, "workspace allocation failed");
        w.capacity = cap;
    }
    *out = &w;
    return HYDRA_PHSP_OK;
}

int release_workspaces() {
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail_hip(e, "hipDeviceSynchronize");
    for (auto& kv : g_ws) {
        if (kv.second.partials) (void)hipFree(kv.second.partials);
        if (kv.second.stats_dev) (void)hipFree(kv.second.stats_dev);
        if (kv.second.mid) (void)hipFree(kv.second.mid);
        if (kv.second.stats_host) (void)hipHostFree(kv.second.stats_host);
    }
    g_ws.clear();
    return HYDRA_PHSP_OK;
}

// ------------------------------------------------------ trigonometric table ----

// (cos, sin)(2 pi k / kTrigSize) for k = 0..kTrigSize-1, evaluated in long double
// and rounded once.  The table lives in a file-scope device array (every GPU
// holds its own copy), uploaded once per device on first use; no allocation.
static __device__ __align__(256) double2 trig_dev[kTrigSize];

constexpr int kMaxDevices = 64;
static std::mutex g_trig_mu;
static double2* g_trig[kMaxDevices]; // per device: address of its trig_dev copy, once uploaded

int trig_table(const double2** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(HYDRA_PHSP_EINVAL, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(g_trig_mu);
    if (g_trig[dev] != nullptr) {
        *out = g_trig[dev];
        return HYDRA_PHSP_OK;
    }
    const long double two_pi = 6.283185307179586476925286766559005768L;
    double2 h[kTrigSize];
    for (int k = 0; k < kTrigSize; ++k) {
        const long double a = two_pi * (long double)k / (long double)kTrigSize;
        h[k].x = (double)cosl(a);
        h[k].y = (double)sinl(a);
    }
    double2* d = nullptr;
    e = hipGetSymbolAddress((void**)&d, HIP_SYMBOL(trig_dev));
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(trig table)");
    e = hipMemcpy(d, h, sizeof(h), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "table upload");
    g_trig[dev] = d;
    *out = d;
    return HYDRA_PHSP_OK;
}

// ------------------------------------------------------- fixed scratch ----

// Device memory of the allocation-free entry point: the stage-1 merge results
// (kMaxGroups) followed by up to kScratchPartials block partials, in one
// file-scope device array.  Each GPU holds its own copy for the life of the
// process; calls on one GPU share it (and race if they overlap).  Host code
// only ever uses the per-device address from hipGetSymbolAddress, never the
// array's name (which on the host is a stand-in, not a device address).
constexpr uint64_t kScratchPartials = 1ull << 20;
static __device__ __align__(256) Moments scratch[kMaxGroups + kScratchPartials];

static std::mutex g_scratch_mu;
static Moments* g_scratch[kMaxDevices]; // per device: address of its scratch copy

// Set-up on first use per device (the device must be current): look up this
// device's scratch address, and make sure its trigonometric table is uploaded.
static int scratch_for_current_device(Moments** out, const double2** trig) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(HYDRA_PHSP_EINVAL, "device index beyond the library's table");
    const int st = trig_table(trig);
    if (st != HYDRA_PHSP_OK) return st;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[dev] == nullptr) {
        Moments* p = nullptr;
        e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return HYDRA_PHSP_OK;
}

// ----------------------------------------------------------------- timing ----

struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool; // created lazily, reused
    size_t used = 0;
};
static Timing g_timing;

// Returns the slot whose events bracket the next launch, or -1 when disabled.
long timing_begin(hipStream_t stream) {
    std::lock_guard<std::mutex> lock(g_timing.mu);
    if (!g_timing.on) return -1;
    if (g_timing.used == g_timing.pool.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return -1;
        if (hipEventCreate(&b) != hipSuccess) {
            (void)hipEventDestroy(a);
            return -1;
        }
        g_timing.pool.emplace_back(a, b);
    }
    const long slot = (long)g_timing.used++;
    if (hipEventRecord(g_timing.pool[slot].first, stream) != hipSuccess) return -1;
    return slot;
}

void timing_end(hipStream_t stream, long slot) {
    if (slot < 0) return;
    std::lock_guard<std::mutex> lock(g_timing.mu);
    (void)hipEventRecord(g_timing.pool[slot].second, stream);
}

// ----------------------------------------------------------------- launch ----

__global__ __launch_bounds__(kStage1Block) void k_merge_stage1(const Moments* parts, uint64_t count,
                                                              Moments* mid) {
    const Moments r = stage1_group(parts, count, blockIdx.x);
    if (threadIdx.x == 0) mid[blockIdx.x] = r;
}

__global__ __launch_bounds__(kStage2Block) void k_merge_stage2(const Moments* mid, uint64_t groups,
                                                              double* stats) {
    stage2_write(mid, groups, stats);
}

static hipError_t launch_by_n(int n, const LaunchSpec& s, const KArgs& a, hipStream_t stream) {
    switch (n) {
    case 2: return launch_phsp<2>(s, a, stream);
    case 3: return launch_phsp<3>(s, a, stream);
    case 4: return launch_phsp<4>(s, a, stream);
    case 5: return launch_phsp<5>(s, a, stream);
    case 6: return launch_phsp<6>(s, a, stream);
    case 7: return launch_phsp<7>(s, a, stream);
    case 8: return launch_phsp<8>(s, a, stream);
    case 9: return launch_phsp<9>(s, a, stream);
    case 10: return launch_phsp<10>(s, a, stream);
    default: return hipErrorInvalidValue;
    }
}

// Events per thread of the single-channel kernels (0 = default per path).  The
// defaults are the fastest of 1, 2 and 4 in two warmed sweeps on MI355X (about
// 10 GB of output per launch, N pions from 10 GeV).  Integration stores
// nothing, so four events per lane amortise the block reduction best.  For FP64
// generation blocks that span 256 or 512 events per column stream their stores
// faster than blocks spanning 1024, which favours one event per lane for N = 3
// (and for per-event parents, which also read) and two for N = 2, 4 and 5;
// from N = 6 the per-event work dominates and four pay off (the top-down levels
// keep one subsystem live, so four events per lane still fit in about 128
// VGPRs).  The mixed path computes the same FP64 events but stores half the
// bytes, so its arithmetic dominates earlier: four events per lane from N = 3.
static std::atomic<int> g_ept_override[3] = {{0}, {0}, {0}}; // read by launches on any thread
// Off the line grid the staged kernel's LDS rounds and barriers change the
// balance: measured the same way, a longer block run pays off for N = 3 (and
// N = 2 with FP32 stores), while from N = 5 the staged kernel, which holds every
// daughter of its events until they are staged, is fastest at one event per
// lane.
static int default_ept(int mode, int n, int pmode, bool staged) {
    const int o = g_ept_override[mode].load(std::memory_order_relaxed);
    if (o > 0) return o;
    if (mode == kIntegrate) return kEptIntegrate;
    if (staged) {
        static const int kStagedFp64[11] = {0, 0, 2, 4, 2, 1, 1, 1, 1, 1, 1};
        static const int kStagedMixed[11] = {0, 0, 4, 4, 2, 1, 1, 1, 1, 1, 1};
        return mode == kMixed ? kStagedMixed[n] : kStagedFp64[n];
    }
    if (pmode == kPerEvent && n <= 3) return 1;
    static const int kMixedTable[11] = {0, 0, 2, 4, 4, 4, 4, 4, 4, 4, 4};
    return mode == kMixed ? kMixedTable[n] : kEptLineFp64[n];
}

int single_channel_ept(int mode, int n, int pmode, bool staged) { return default_ept(mode, n, pmode, staged); }

// Launch shape of a single-channel call: events per thread, block count and
// kernel form (direct or staged stores).
struct SingleShape {
    int ept;
    uint64_t blocks;
    bool staged;
};

static int single_shape(int n, int pmode, uint64_t nevents, int mode, const void* out, uint64_t ld,
                        const double* weights, int ept_override, SingleShape* sh) {
    // Columns on the 128-byte line grid take the direct-store kernel; any other
    // layout the staged one (whole-line writes through LDS).
    const uint64_t elem = mode == kMixed ? sizeof(float) : sizeof(double);
    const bool aligned = (uintptr_t)out % kLineBytes == 0 && (ld * elem) % kLineBytes == 0 &&
                         (uintptr_t)weights % kLineBytes == 0;
    sh->staged = mode != kIntegrate && !aligned;
    sh->ept = ept_override > 0 ? ept_override : default_ept(mode, n, pmode, sh->staged);
    const uint64_t per_block = (uint64_t)kBlock * (uint64_t)sh->ept;
    sh->blocks = ceil_div(nevents, per_block);
    if (sh->blocks > 0xFFFFFFFFull / (uint64_t)kBlock)
        return fail(HYDRA_PHSP_EINVAL, "nevents too large for one launch (more than 2^32 - 1 threads)");
    return HYDRA_PHSP_OK;
}

// The launches of one single-channel call with its block partials at `partials`
// and the stage-1 merge results at `mid` (both large enough for sh.blocks).
static int enqueue_single(const Channel& ch, int n, int pmode, const Frame* frame, const double* parent_dev,
                          uint64_t ld_parent, uint64_t nevents, uint64_t seed, uint32_t sid, uint64_t offset,
                          int mode, void* out, uint64_t ld, double* weights, double* stats_dev,
                          hipStream_t stream, const SingleShape& sh, Moments* partials, Moments* mid,
                          const double2* trig, bool timed);

int run_single(const Channel& ch, int n, int pmode, const Frame* frame, const double* parent_dev,
               uint64_t ld_parent, uint64_t nevents, uint64_t seed, uint32_t sid, uint64_t offset,
               int mode, void* out, uint64_t ld, double* weights, double* stats_dev,
               hipStream_t stream, int ept_override) {
    SingleShape sh;
    int st = single_shape(n, pmode, nevents, mode, out, ld, weights, ept_override, &sh);
    if (st != HYDRA_PHSP_OK) return st;
    Workspace* ws = nullptr;
    st = workspace_for(stream, sh.blocks, &ws);
    if (st != HYDRA_PHSP_OK) return st;
    const double2* trig = nullptr;
    st = trig_table(&trig);
    if (st != HYDRA_PHSP_OK) return st;
    return enqueue_single(ch, n, pmode, frame, parent_dev, ld_parent, nevents, seed, sid, offset, mode, out, ld,
                          weights, stats_dev, stream, sh, ws->partials, ws->mid, trig, true);
}

static int merge_partials_into(hipStream_t stream, const Moments* partials, uint64_t blocks, Moments* mid,
                               double* stats_dev);

static int enqueue_single(const Channel& ch, int n, int pmode, const Frame* frame, const double* parent_dev,
                          uint64_t ld_parent, uint64_t nevents, uint64_t seed, uint32_t sid, uint64_t offset,
                          int mode, void* out, uint64_t ld, double* weights, double* stats_dev,
                          hipStream_t stream, const SingleShape& sh, Moments* partials, Moments* mid,
                          const double2* trig, bool timed) {
    const uint64_t blocks = sh.blocks;
    if (blocks > 0) {
        KArgs a;
        std::memset(&a, 0, sizeof(a));
        a.ch = ch;
        if (frame) a.frame = *frame;
        a.parent = parent_dev;
        a.ld_parent = ld_parent;
        a.inv_M = 1.0 / ch.M;
        a.nevents = nevents;
        a.event_offset = offset;
        a.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
        a.k1 = (uint32_t)(seed >> 32);
        a.sid = sid;
        a.out = out;
        a.ld = ld;
        a.weights = weights;
        a.partials = partials;
        a.trig = trig;
        LaunchSpec s{pmode, mode, sh.ept, blocks, sh.staged};
        const long slot = timed ? timing_begin(stream) : -1;
        hipError_t e = launch_by_n(n, s, a, stream);
        timing_end(stream, slot);
        if (e != hipSuccess) return fail_hip(e, "phase-space kernel launch");
    }
    if (stats_dev != nullptr) return merge_partials_into(stream, partials, blocks, mid, stats_dev);
    return HYDRA_PHSP_OK;
}

int block_partials(hipStream_t stream, uint64_t blocks, Moments** partials) {
    Workspace* ws = nullptr;
    const int st = workspace_for(stream, blocks, &ws);
    if (st == HYDRA_PHSP_OK) *partials = ws->partials;
    return st;
}

int merge_partials(hipStream_t stream, const Moments* partials, uint64_t blocks, double* stats_dev) {
    Workspace* ws = nullptr;
    const int st = workspace_for(stream, blocks, &ws);
    if (st != HYDRA_PHSP_OK) return st;
    return merge_partials_into(stream, partials, blocks, ws->mid, stats_dev);
}

static int merge_partials_into(hipStream_t stream, const Moments* partials, uint64_t blocks, Moments* mid,
                               double* stats_dev) {
    const uint64_t groups = stage1_groups(blocks);
    hipLaunchKernelGGL(k_merge_stage1, dim3((unsigned)groups), dim3(kStage1Block), 0, stream, partials, blocks,
                       mid);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "merge kernel launch");
    hipLaunchKernelGGL(k_merge_stage2, dim3(1), dim3(kStage2Block), 0, stream, (const Moments*)mid, groups,
                       stats_dev);
    e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "merge kernel launch");
    return HYDRA_PHSP_OK;
}

static int generate_common(double M, const double* masses, int n, const double* parent_p4_host,
                           const double* parent_p4_dev, uint64_t ld_parent, uint64_t nevents,
                           uint64_t seed, uint32_t sid, uint64_t offset, void* out, uint64_t ld,
                           double* weights, double* stats_dev, void* stream, int mode, bool noalloc = false) {
    Channel ch;
    int st = make_channel(M, masses, n, &ch);
    if (st != HYDRA_PHSP_OK) return st;
    if (nevents > 0 && (out == nullptr || weights == nullptr))
        return fail(HYDRA_PHSP_EINVAL, "p4_out_dev and weights_dev are required");
    if (ld < nevents) return fail(HYDRA_PHSP_EINVAL, "ld must be >= nevents");
    const uintptr_t elem = mode == kMixed ? sizeof(float) : sizeof(double);
    if ((uintptr_t)out % elem != 0 || (uintptr_t)weights % sizeof(double) != 0 ||
        (uintptr_t)stats_dev % sizeof(double) != 0 || (uintptr_t)parent_p4_dev % sizeof(double) != 0)
        return fail(HYDRA_PHSP_EINVAL, "device pointers must be aligned to their element size");
    if (parent_p4_host != nullptr && parent_p4_dev != nullptr)
        return fail(HYDRA_PHSP_EINVAL, "give at most one of parent_p4_host and parent_p4_dev");
    int pmode = kAtRest;
    Frame frame;
    std::memset(&frame, 0, sizeof(frame));
    if (parent_p4_host != nullptr) {
        st = make_frame(M, parent_p4_host, &frame);
        if (st != HYDRA_PHSP_OK) return st;
        pmode = kBroadcast;
    } else if (parent_p4_dev != nullptr) {
        if (ld_parent < nevents) return fail(HYDRA_PHSP_EINVAL, "ld_parent must be >= nevents");
        pmode = kPerEvent;
    }
    if (!noalloc)
        return run_single(ch, n, pmode, &frame, parent_p4_dev, ld_parent, nevents, seed, sid, offset, mode,
                          out, ld, weights, stats_dev, (hipStream_t)stream, 0);
    // Same launches and kernels, with the partials and merge results in the
    // fixed scratch array instead of the per-stream workspace; nothing needs
    // clearing (every block writes its partial, every group its merge result).
    SingleShape sh;
    st = single_shape(n, pmode, nevents, mode, out, ld, weights, 0, &sh);
    if (st != HYDRA_PHSP_OK) return st;
    if (sh.blocks > kScratchPartials)
        return fail(HYDRA_PHSP_EINVAL, "nevents too large for hydra_phsp_generate_noalloc: more than " +
                                           std::to_string(kScratchPartials) + " blocks of " +
                                           std::to_string(kBlock * sh.ept) + " events");
    Moments* fixed = nullptr;
    const double2* trig = nullptr;
    st = scratch_for_current_device(&fixed, &trig);
    if (st != HYDRA_PHSP_OK) return st;
    return enqueue_single(ch, n, pmode, &frame, parent_p4_dev, ld_parent, nevents, seed, sid, offset, mode, out,
                          ld, weights, stats_dev, (hipStream_t)stream, sh, fixed + kMaxGroups, fixed, trig, false);
}

} // namespace hphsp

using namespace hphsp;

extern "C" {

int hydra_phsp_generate(double parent_mass, const double* masses_host, int n_daughters,
                        const double* parent_p4_host, const double* parent_p4_dev, uint64_t ld_parent,
                        uint64_t nevents, uint64_t seed, uint32_t stream_id, uint64_t event_offset,
                        double* p4_out_dev, uint64_t ld, double* weights_dev, double* stats_dev,
                        void* stream) {
    MarkerRange marker("hydra_phsp_generate");
    return generate_common(parent_mass, masses_host, n_daughters, parent_p4_host, parent_p4_dev,
                           ld_parent, nevents, seed, stream_id, event_offset, p4_out_dev, ld,
                           weights_dev, stats_dev, stream, kFp64);
}

int hydra_phsp_generate_noalloc(double parent_mass, const double* masses_host, int n_daughters,
                                const double* parent_p4_host, const double* parent_p4_dev, uint64_t ld_parent,
                                uint64_t nevents, uint64_t seed, uint32_t stream_id, uint64_t event_offset,
                                double* p4_out_dev, uint64_t ld, double* weights_dev, double* stats_dev,
                                void* stream) {
    return generate_common(parent_mass, masses_host, n_daughters, parent_p4_host, parent_p4_dev,
                           ld_parent, nevents, seed, stream_id, event_offset, p4_out_dev, ld,
                           weights_dev, stats_dev, stream, kFp64, true);
}

int hydra_phsp_generate_mixed(double parent_mass, const double* masses_host, int n_daughters,
                              const double* parent_p4_host, const double* parent_p4_dev,
                              uint64_t ld_parent, uint64_t nevents, uint64_t seed, uint32_t stream_id,
                              uint64_t event_offset, float* p4_out_dev, uint64_t ld,
                              double* weights_dev, double* stats_dev, void* stream) {
    MarkerRange marker("hydra_phsp_generate_mixed");
    return generate_common(parent_mass, masses_host, n_daughters, parent_p4_host, parent_p4_dev,
                           ld_parent, nevents, seed, stream_id, event_offset, p4_out_dev, ld,
                           weights_dev, stats_dev, stream, kMixed);
}

int hydra_phsp_integrate_async(double parent_mass, const double* masses_host, int n_daughters,
                               uint64_t nevents, uint64_t seed, uint32_t stream_id,
                               uint64_t event_offset, double* stats_dev, void* stream) {
    MarkerRange marker("hydra_phsp_integrate_async");
    Channel ch;
    int st = make_channel(parent_mass, masses_host, n_daughters, &ch);
    if (st != HYDRA_PHSP_OK) return st;
    if (stats_dev == nullptr) return fail(HYDRA_PHSP_EINVAL, "stats_dev is NULL");
    return run_single(ch, n_daughters, kAtRest, nullptr, nullptr, 0, nevents, seed, stream_id,
                      event_offset, kIntegrate, nullptr, 0, nullptr, stats_dev, (hipStream_t)stream, 0);
}

int hydra_phsp_integrate(double parent_mass, const double* masses_host, int n_daughters,
                         uint64_t nevents, uint64_t seed, uint32_t stream_id, uint64_t event_offset,
                         double* mean_host, double* sigma_host, void* stream) {
    MarkerRange marker("hydra_phsp_integrate");
    Channel ch;
    int st = make_channel(parent_mass, masses_host, n_daughters, &ch);
    if (st != HYDRA_PHSP_OK) return st;
    if (mean_host == nullptr || sigma_host == nullptr)
        return fail(HYDRA_PHSP_EINVAL, "mean_host and sigma_host are required");
    if (nevents < 2) return fail(HYDRA_PHSP_EINVAL, "integrate needs nevents >= 2");
    hipStream_t s = (hipStream_t)stream;
    Workspace* ws = nullptr;
    st = workspace_for(s, 1, &ws);
    if (st != HYDRA_PHSP_OK) return st;
    st = run_single(ch, n_daughters, kAtRest, nullptr, nullptr, 0, nevents, seed, stream_id, event_offset,
                    kIntegrate, nullptr, 0, nullptr, ws->stats_dev, s, 0);
    if (st != HYDRA_PHSP_OK) return st;
    hipError_t e = hipMemcpyAsync(ws->stats_host, ws->stats_dev, sizeof(double) * HYDRA_PHSP_STATS,
                                  hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    *mean_host = ws->stats_host[1];
    *sigma_host = ws->stats_host[3];
    return HYDRA_PHSP_OK;
}

const char* hydra_phsp_strerror(int status) {
    switch (status) {
    case HYDRA_PHSP_OK: return "ok";
    case HYDRA_PHSP_EINVAL: return "invalid argument";
    case HYDRA_PHSP_EKINEMATICS: return "kinematically forbidden decay (parent mass <= sum of daughter masses)";
    case HYDRA_PHSP_ENOMEM: return "out of memory";
    case HYDRA_PHSP_EDEVICE: return "HIP device error";
    case HYDRA_PHSP_EAGAIN: return "result not ready";
    case HYDRA_PHSP_ENOTFOUND: return "unknown request id";
    default: return "unknown status";
    }
}

const char* hydra_phsp_last_error(void) { return t_last_error.c_str(); }

int hydra_phsp_abi_version(void) { return HYDRA_PHSP_ABI_VERSION; }

int hydra_phsp_stats_merge(const double* a_host, const double* b_host, double* out_host) {
    if (a_host == nullptr || b_host == nullptr || out_host == nullptr)
        return fail(HYDRA_PHSP_EINVAL, "stats records must not be NULL");
    const double* rec[2] = {a_host, b_host};
    for (const double* r : rec) {
        if (!std::isfinite(r[0]) || r[0] < 0.0 || r[0] != std::floor(r[0]))
            return fail(HYDRA_PHSP_EINVAL, "stats n must be a finite non-negative integer");
        if (!std::isfinite(r[1]) || !std::isfinite(r[2]) || r[2] < 0.0)
            return fail(HYDRA_PHSP_EINVAL, "stats mean and M2 must be finite, M2 >= 0");
    }
    const Moments m = merge(Moments{a_host[0], a_host[1], a_host[2]}, Moments{b_host[0], b_host[1], b_host[2]});
    out_host[0] = m.n;
    out_host[1] = m.mean;
    out_host[2] = m.m2;
    out_host[3] = m.n >= 2.0 ? std::sqrt(m.m2 / ((m.n - 1.0) * m.n)) : 0.0;
    return HYDRA_PHSP_OK;
}

int hydra_phsp_release(void) {
    const int a = release_batch_slots();
    const int b = release_workspaces(); // synchronizes the device first
    const int c = release_unweight_workspaces();
    const int d = release_vegas_workspaces();
    return a != HYDRA_PHSP_OK ? a : (b != HYDRA_PHSP_OK ? b : (c != HYDRA_PHSP_OK ? c : d));
}

int hydra_phsp_set_events_per_thread(int path, int ept) {
    if (path < 0 || path > 2) return fail(HYDRA_PHSP_EINVAL, "path must be 0, 1 or 2");
    if (ept != 0 && ept != 1 && ept != 2 && ept != 4) return fail(HYDRA_PHSP_EINVAL, "ept must be 0, 1, 2 or 4");
    g_ept_override[path].store(ept, std::memory_order_relaxed);
    return HYDRA_PHSP_OK;
}

int hydra_phsp_events_per_thread(int path, int n_daughters, int flags) {
    if (path < 0 || path > 2) return fail(HYDRA_PHSP_EINVAL, "path must be 0, 1 or 2");
    if (n_daughters < 2 || n_daughters > HYDRA_PHSP_NMAX)
        return fail(HYDRA_PHSP_EINVAL, "n_daughters must be in [2, HYDRA_PHSP_NMAX]");
    if (flags & ~(HYDRA_PHSP_EPT_PER_EVENT_PARENTS | HYDRA_PHSP_EPT_OFF_LINE_GRID))
        return fail(HYDRA_PHSP_EINVAL, "flags must combine HYDRA_PHSP_EPT_PER_EVENT_PARENTS and "
                                       "HYDRA_PHSP_EPT_OFF_LINE_GRID");
    return default_ept(path, n_daughters, (flags & HYDRA_PHSP_EPT_PER_EVENT_PARENTS) ? kPerEvent : kAtRest,
                       path != kIntegrate && (flags & HYDRA_PHSP_EPT_OFF_LINE_GRID) != 0);
}

int hydra_phsp_timing_enable(int on) {
    std::lock_guard<std::mutex> lock(g_timing.mu);
    g_timing.on = on != 0;
    return HYDRA_PHSP_OK;
}

int hydra_phsp_timing_reset(void) {
    std::lock_guard<std::mutex> lock(g_timing.mu);
    g_timing.used = 0;
    return HYDRA_PHSP_OK;
}

int hydra_phsp_timing_read(double* total_ms_host, uint64_t* launches_host) {
    if (total_ms_host == nullptr || launches_host == nullptr)
        return fail(HYDRA_PHSP_EINVAL, "timing_read needs two host pointers");
    std::lock_guard<std::mutex> lock(g_timing.mu);
    double total = 0.0;
    for (size_t i = 0; i < g_timing.used; ++i) {
        hipError_t e = hipEventSynchronize(g_timing.pool[i].second);
        if (e != hipSuccess) return fail_hip(e, "hipEventSynchronize");
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, g_timing.pool[i].first, g_timing.pool[i].second);
        if (e != hipSuccess) return fail_hip(e, "hipEventElapsedTime");
        total += (double)ms;
    }
    *total_ms_host = total;
    *launches_host = (uint64_t)g_timing.used;
    return HYDRA_PHSP_OK;
}

int hydra_phsp_selftest_sortnet(void) {
    bool ok = true;
    auto check = [&](auto tag) {
        constexpr int K = decltype(tag)::value;
        for (int bits = 0; bits < (1 << K); ++bits) {
            int v[K > 0 ? K : 1];
            for (int i = 0; i < K; ++i) v[i] = (bits >> i) & 1;
            sortnet_sort<K, int>(v);
            for (int i = 0; i + 1 < K; ++i)
                if (v[i] > v[i + 1]) ok = false;
        }
    };
    check(std::integral_constant<int, 1>{});
    check(std::integral_constant<int, 2>{});
    check(std::integral_constant<int, 3>{});
    check(std::integral_constant<int, 4>{});
    check(std::integral_constant<int, 5>{});
    check(std::integral_constant<int, 6>{});
    check(std::integral_constant<int, 7>{});
    check(std::integral_constant<int, 8>{});
    return ok ? HYDRA_PHSP_OK : fail(HYDRA_PHSP_EINVAL, "sorting network self-test failed");
}

} // extern "C"

// phsp_unweight_api.hip -- C ABI of the unweighted (hit-or-miss) path: the
// per-stream workspace, the scan of the per-segment counts and the launch
// sequence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>

#include "hydra_phsp.h"
#include "hydra_phsp_model.h"
#include "hydra_phsp_unweight.h"
#include "phsp_api_internal.hpp"
#include "phsp_unweight.hpp"

namespace hphsp {

constexpr int kScanBlock = 256;   // counts scanned per block of the partial scan
constexpr int kScanTop = 1024;    // threads of the single-block scan of the partial sums

__global__ void k_unw_set(double* __restrict__ w_max, double value) {
    if (threadIdx.x == 0) *w_max = value;
}

// Inclusive scan of one value per thread across a block of BLOCK threads
// (wave shuffles, then the wave totals through LDS).
template <int BLOCK>
__device__ __forceinline__ uint64_t block_inclusive_scan(uint64_t v, uint64_t* sm) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t o = __shfl_up(v, off, 64);
        if (lane >= off) v += o;
    }
    if (lane == 63) sm[wave] = v;
    __syncthreads();
    uint64_t add = 0;
    for (int w = 0; w < wave; ++w) add += sm[w];
    __syncthreads();
    return v + add;
}

// Stage 1: kept and over-bound trials of each group of kScanBlock segments, for
// the groups of one chunk (segments [seg_lo, segments), seg_lo a multiple of
// kScanBlock; block b takes group g = seg_lo / kScanBlock + b).
__global__ __launch_bounds__(kScanBlock) void k_unw_scan_partial(const uint2* __restrict__ counts, uint64_t seg_lo,
                                                                 uint64_t segments, uint64_t* __restrict__ sums,
                                                                 uint64_t* __restrict__ over_sums) {
    __shared__ uint64_t sm[kScanBlock / 64];
    const uint64_t g = seg_lo / kScanBlock + blockIdx.x;
    const uint64_t i = g * kScanBlock + threadIdx.x;
    const uint64_t v = i < segments ? counts[i].x : 0u;
    const uint64_t inc = block_inclusive_scan<kScanBlock>(v, sm);
    if (threadIdx.x == kScanBlock - 1) sums[g] = inc;
    uint64_t o = i < segments ? counts[i].y : 0u;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) o += __shfl_xor(o, off, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = o; // the scan's last read of sm was before its barrier
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
#pragma unroll
        for (int w = 0; w < kScanBlock / 64; ++w) t += sm[w];
        over_sums[g] = t;
    }
}

// Stage 2 (one block per chunk): exclusive prefix of the chunk's group sums, in
// place, starting from the kept total of the chunks before it; that total plus
// the chunk's into chunk_kept[chunk], the chunk's over-bound trials into
// chunk_over[chunk].  The last chunk also writes the totals (kept, over-bound)
// into the caller's counts and the bound applied into the caller's w_max output
// when asked.
__global__ __launch_bounds__(kScanTop) void k_unw_scan_top(uint64_t* __restrict__ sums, uint64_t groups,
                                                           const uint64_t* __restrict__ over_sums,
                                                           uint64_t* __restrict__ chunk_kept,
                                                           uint64_t* __restrict__ chunk_over, uint32_t chunk,
                                                           uint32_t last_chunk, uint64_t* __restrict__ totals,
                                                           const double* __restrict__ w_max,
                                                           double* __restrict__ w_max_out) {
    __shared__ uint64_t sm[kScanTop / 64];
    __shared__ uint64_t last;
    uint64_t carry = chunk > 0 ? chunk_kept[chunk - 1] : 0;
    for (uint64_t b0 = 0; b0 < groups; b0 += kScanTop) {
        const uint64_t i = b0 + threadIdx.x;
        const uint64_t v = i < groups ? sums[i] : 0u;
        const uint64_t inc = block_inclusive_scan<kScanTop>(v, sm);
        if (i < groups) sums[i] = carry + inc - v;
        if (threadIdx.x == kScanTop - 1) last = inc; // this chunk's total
        __syncthreads();
        carry += last;
        __syncthreads();
    }
    // over-bound trials: a plain sum of the group sums (order-free for integers)
    uint64_t over = 0;
    for (uint64_t i = threadIdx.x; i < groups; i += kScanTop) over += over_sums[i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) over += __shfl_xor(over, off, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = over;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t o = 0;
        for (int w = 0; w < kScanTop / 64; ++w) o += sm[w];
        chunk_kept[chunk] = carry;
        chunk_over[chunk] = o;
        if (last_chunk) {
            for (uint32_t c = 0; c < chunk; ++c) o += chunk_over[c];
            totals[0] = carry;
            totals[1] = o;
            if (w_max_out != nullptr) *w_max_out = *w_max;
        }
    }
}

// Stage 3: each segment's offset = its group's prefix + the kept counts of the
// earlier segments of the group; the segment whose run [offset, offset + kept)
// holds a range start r * kUnwRange is recorded as that range's first segment
// (a run is at most kUnwSeg long, so it holds at most kUnwSeg / kUnwRange
// starts, and the runs tile [0, kept), so every range start has its segment).
static_assert(kUnwSeg % kUnwRange == 0, "whole ranges per segment");
// Segments [seg_lo, segments) of one chunk; seg_lo is a multiple of kScanBlock,
// so block b scans group seg_lo / kScanBlock + b.
__global__ __launch_bounds__(kScanBlock) void k_unw_scan_finish(const uint2* __restrict__ counts, uint64_t seg_lo,
                                                                uint64_t segments, const uint64_t* __restrict__ sums,
                                                                uint64_t* __restrict__ offsets,
                                                                uint64_t* __restrict__ range_seg) {
    __shared__ uint64_t sm[kScanBlock / 64];
    const uint64_t i = seg_lo + (uint64_t)blockIdx.x * kScanBlock + threadIdx.x;
    const uint64_t v = i < segments ? counts[i].x : 0u;
    const uint64_t inc = block_inclusive_scan<kScanBlock>(v, sm);
    if (i < segments) {
        const uint64_t o = sums[seg_lo / kScanBlock + blockIdx.x] + inc - v;
        offsets[i] = o;
        for (uint64_t r = (o + kUnwRange - 1) / kUnwRange; r * kUnwRange < o + v; ++r) range_seg[r] = i;
    }
}

// Chunks of the count-scan-write pipeline: at most kMaxChunks, each of whole
// scan groups (kScanBlock segments, 262144 trials).
constexpr int kMaxChunks = 16;
constexpr int kDefaultChunks = 4;      // acceptance against the weight alone
constexpr int kDefaultChunksModel = 1; // against a model: few trials kept, so little store work to overlap
// A model's trial values are kept between the max and count passes for at most
// this many trials (8 bytes each: 2 GiB); larger calls recompute them.
constexpr uint64_t kMaxStoredValues = 1ull << 28;
std::atomic<int> g_chunks_override{0};

namespace {

struct UnwWorkspace {
    uint2* counts = nullptr;       // [segments]
    uint64_t* offsets = nullptr;   // [segments]
    uint64_t* range_seg = nullptr; // first segment of each write-pass range: [segments * kUnwSeg / kUnwRange]
    uint64_t* masks = nullptr;     // [segments * kUnwSegWords], allocated when outputs are asked for
    double* values = nullptr;      // [value_capacity] trial values of a model (sample-maximum calls)
    uint64_t* sums = nullptr;      // [groups] kept trials per group of kScanBlock segments
    uint64_t* over_sums = nullptr; // [groups] over-bound trials per group
    double* w_max = nullptr;
    uint64_t* chunk_kept = nullptr; // [kMaxChunks] kept trials of chunks 0..k together
    uint64_t* chunk_over = nullptr; // [kMaxChunks] over-bound trials per chunk
    uint64_t capacity = 0;         // segments
    uint64_t mask_capacity = 0;    // segments
    uint64_t value_capacity = 0;   // trials
};

std::mutex g_unw_mu;
std::map<std::pair<int, hipStream_t>, UnwWorkspace> g_unw_ws;

void free_ws(UnwWorkspace& w) {
    if (w.counts) (void)hipFree(w.counts);
    if (w.offsets) (void)hipFree(w.offsets);
    if (w.range_seg) (void)hipFree(w.range_seg);
    if (w.masks) (void)hipFree(w.masks);
    if (w.sums) (void)hipFree(w.sums);
    if (w.over_sums) (void)hipFree(w.over_sums);
    if (w.w_max) (void)hipFree(w.w_max);
    if (w.chunk_kept) (void)hipFree(w.chunk_kept);
    if (w.chunk_over) (void)hipFree(w.chunk_over);
    if (w.values) (void)hipFree(w.values);
    w.values = nullptr;
    w.value_capacity = 0;
    w.counts = nullptr;
    w.offsets = w.range_seg = w.masks = w.sums = w.over_sums = w.chunk_kept = w.chunk_over = nullptr;
    w.w_max = nullptr;
    w.capacity = w.mask_capacity = 0;
}

int unw_workspace(hipStream_t stream, uint64_t segments, bool masks, uint64_t values, UnwWorkspace** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_unw_mu);
    UnwWorkspace& w = g_unw_ws[std::make_pair(dev, stream)];
    if (masks && segments > w.mask_capacity) {
        uint64_t cap = w.mask_capacity ? w.mask_capacity : 4096;
        while (cap < segments) cap *= 2;
        if (w.masks) (void)hipFree(w.masks); // waits for the device: no queued kernel still uses it
        w.masks = nullptr;
        w.mask_capacity = 0;
        if (hipMalloc(&w.masks, sizeof(uint64_t) * kUnwSegWords * cap) != hipSuccess) {
            w.masks = nullptr;
            return fail(HYDRA_PHSP_ENOMEM, "unweighting mask allocation failed");
        }
        w.mask_capacity = cap;
    }
    if (values > w.value_capacity) {
        uint64_t cap = w.value_capacity ? w.value_capacity : (1ull << 20);
        while (cap < values) cap *= 2;
        if (w.values) (void)hipFree(w.values); // waits for the device: no queued kernel still uses it
        w.values = nullptr;
        w.value_capacity = 0;
        if (hipMalloc(&w.values, sizeof(double) * cap) != hipSuccess) {
            w.values = nullptr;
            return fail(HYDRA_PHSP_ENOMEM, "unweighting value allocation failed");
        }
        w.value_capacity = cap;
    }
    if (w.w_max == nullptr || segments > w.capacity) {
        uint64_t cap = w.capacity ? w.capacity : 4096;
        while (cap < segments) cap *= 2;
        uint64_t* keep_masks = w.masks;
        const uint64_t keep_mask_cap = w.mask_capacity;
        double* keep_values = w.values;
        const uint64_t keep_value_cap = w.value_capacity;
        w.masks = nullptr; // kept across the regrowth of the other buffers
        w.values = nullptr;
        free_ws(w); // hipFree waits for the device, so no queued kernel still uses it
        w.masks = keep_masks;
        w.mask_capacity = keep_mask_cap;
        w.values = keep_values;
        w.value_capacity = keep_value_cap;
        const uint64_t groups = (cap + kScanBlock - 1) / kScanBlock;
        bool ok = hipMalloc(&w.counts, sizeof(uint2) * cap) == hipSuccess &&
                  hipMalloc(&w.offsets, sizeof(uint64_t) * cap) == hipSuccess &&
                  hipMalloc(&w.range_seg, sizeof(uint64_t) * cap * (kUnwSeg / kUnwRange)) == hipSuccess &&
                  hipMalloc(&w.sums, sizeof(uint64_t) * groups) == hipSuccess &&
                  hipMalloc(&w.over_sums, sizeof(uint64_t) * groups) == hipSuccess &&
                  hipMalloc(&w.w_max, sizeof(double)) == hipSuccess &&
                  hipMalloc(&w.chunk_kept, sizeof(uint64_t) * kMaxChunks) == hipSuccess &&
                  hipMalloc(&w.chunk_over, sizeof(uint64_t) * kMaxChunks) == hipSuccess;
        if (!ok) {
            free_ws(w);
            return fail(HYDRA_PHSP_ENOMEM, "unweighting workspace allocation failed");
        }
        w.capacity = cap;
    }
    *out = &w;
    return HYDRA_PHSP_OK;
}

template <int N>
hipError_t launch_pass(int pass, const UnwLaunch& L, hipStream_t s) {
    switch (pass) {
    case 0: return launch_unw_max<N>(L, s);
    case 1: return launch_unw_count<N>(L, s);
    case 2: return launch_unw_write<N>(L, s);
    default: return launch_unw_write_count<N>(L, s);
    }
}

hipError_t launch_pass_n(int n, int pass, const UnwLaunch& L, hipStream_t s) {
    switch (n) {
    case 2: return launch_pass<2>(pass, L, s);
    case 3: return launch_pass<3>(pass, L, s);
    case 4: return launch_pass<4>(pass, L, s);
    case 5: return launch_pass<5>(pass, L, s);
    case 6: return launch_pass<6>(pass, L, s);
    case 7: return launch_pass<7>(pass, L, s);
    case 8: return launch_pass<8>(pass, L, s);
    case 9: return launch_pass<9>(pass, L, s);
    case 10: return launch_pass<10>(pass, L, s);
    default: return hipErrorInvalidValue;
    }
}

} // namespace

int release_unweight_workspaces() {
    std::lock_guard<std::mutex> lock(g_unw_mu);
    for (auto& kv : g_unw_ws) free_ws(kv.second);
    g_unw_ws.clear();
    return HYDRA_PHSP_OK;
}

} // namespace hphsp

using namespace hphsp;

namespace hphsp {
namespace {

// What the trials are accepted against (see UnwArgs): the weight, the built-in
// Breit-Wigner model, or a user model's run-time kernels.
struct UnwIntensity {
    int kind = 0; // 0 weight, 1 Breit-Wigner, 2 user
    BwFactors bw{};
    RtcKernel* user = nullptr;
    double upar[HYDRA_PHSP_USER_PARAMS] = {};
};

int unweighted_run(const Channel& ch, int n_daughters, const double* parent_p4_host, uint64_t ntrials, uint64_t seed,
                   uint32_t stream_id, uint64_t event_offset, double w_max, double* p4_out_dev, uint64_t ld,
                   uint64_t* index_out_dev, uint64_t* counts_dev, double* w_max_dev, void* stream,
                   const UnwIntensity& inten) {
    if (!(w_max >= 0.0) || w_max > 1.7976931348623157e308)
        return fail(HYDRA_PHSP_EINVAL, "w_max must be finite and >= 0 (0: the largest trial value)");
    if (counts_dev == nullptr) return fail(HYDRA_PHSP_EINVAL, "counts_dev is required");
    if ((p4_out_dev != nullptr || index_out_dev != nullptr) && ld == 0)
        return fail(HYDRA_PHSP_EINVAL, "ld (the capacity in events) must be >= 1 when outputs are given");
    if ((uintptr_t)p4_out_dev % sizeof(double) != 0 || (uintptr_t)index_out_dev % sizeof(uint64_t) != 0 ||
        (uintptr_t)counts_dev % sizeof(uint64_t) != 0 || (uintptr_t)w_max_dev % sizeof(double) != 0)
        return fail(HYDRA_PHSP_EINVAL, "device pointers must be aligned to their element size");
    Frame frame;
    std::memset(&frame, 0, sizeof(frame));
    int pmode = kAtRest;
    int st = HYDRA_PHSP_OK;
    if (parent_p4_host != nullptr) {
        st = make_frame(ch.M, parent_p4_host, &frame);
        if (st != HYDRA_PHSP_OK) return st;
        pmode = kBroadcast;
    }
    const uint64_t max_blocks = ceil_div(ntrials, (uint64_t)kBlock * (uint64_t)kUnwEpt);
    const uint64_t segments = ceil_div(ntrials, (uint64_t)kUnwSeg);
    const bool outputs = p4_out_dev != nullptr || index_out_dev != nullptr;
    // Chunks of whole scan groups; without outputs there is no write pass to
    // overlap, so one chunk.
    const uint64_t groups = ceil_div(segments, (uint64_t)kScanBlock);
    const int want_chunks = g_chunks_override.load(std::memory_order_relaxed);
    // (a user model's count kernel is compiled at run time, without a fused form)
    const int default_chunks = inten.kind == 0 ? kDefaultChunks : kDefaultChunksModel;
    const uint64_t chunks_req =
        outputs && inten.kind != 2 ? (uint64_t)(want_chunks > 0 ? want_chunks : default_chunks) : 1;
    const uint64_t chunk_groups = std::max<uint64_t>(ceil_div(groups, chunks_req), 1);
    const uint64_t chunk_segs = chunk_groups * kScanBlock;
    const uint64_t nchunks = std::max<uint64_t>(ceil_div(segments, chunk_segs), 1);
    // count pass: one wave per segment; write pass: one wave per range of output
    // positions a chunk can settle (its trials plus the partial range carried in)
    const uint64_t blocks = ceil_div(std::min(segments, chunk_segs), (uint64_t)kUnwSegPerBlock);
    const uint64_t write_ranges =
        outputs ? std::min(ceil_div(std::min(ntrials, chunk_segs * (uint64_t)kUnwSeg), (uint64_t)kUnwRange) + 1,
                           ceil_div(ld, (uint64_t)kUnwRange))
                : 0;
    const uint64_t write_blocks = ceil_div(write_ranges, (uint64_t)kUnwSegPerBlock);
    // fused pass: a wave per output range of chunk k or per segment of chunk k + 1
    const uint64_t fused_blocks =
        nchunks > 1 ? ceil_div(std::max(write_ranges, chunk_segs), (uint64_t)kUnwSegPerBlock) : 0;
    if (max_blocks > 0xFFFFFFFFull / (uint64_t)kBlock || blocks > 0xFFFFFFFFull / (uint64_t)kBlock ||
        write_blocks > 0xFFFFFFFFull / (uint64_t)kBlock || fused_blocks > 0xFFFFFFFFull / (uint64_t)kBlock)
        return fail(HYDRA_PHSP_EINVAL, "ntrials too large for one launch (more than 2^32 - 1 threads)");
    hipFunction_t user_max = nullptr, user_count = nullptr;
    if (inten.kind == 2) {
        st = rtc_function(inten.user, kUserModelUnwMax, &user_max);
        if (st == HYDRA_PHSP_OK) st = rtc_function(inten.user, kUserModelUnwCount, &user_count);
        if (st != HYDRA_PHSP_OK) return st;
    }

    hipStream_t s = (hipStream_t)stream;
    UnwWorkspace* ws = nullptr;
    // a model's values (the full kinematics of every trial) are computed once for
    // the max pass and the count pass, when no bound is given
    const bool store_values = inten.kind != 0 && w_max == 0.0 && ntrials > 0 && ntrials <= kMaxStoredValues;
    st = unw_workspace(s, std::max<uint64_t>(segments, 1), outputs, store_values ? ntrials : 0, &ws);
    if (st != HYDRA_PHSP_OK) return st;
    const double2* trig = nullptr;
    st = trig_table(&trig);
    if (st != HYDRA_PHSP_OK) return st;

    UnwLaunch L;
    std::memset(&L, 0, sizeof(L));
    L.u.a.ch = ch;
    L.u.a.frame = frame;
    L.u.a.inv_M = 1.0 / ch.M;
    L.u.a.nevents = ntrials;
    L.u.a.event_offset = event_offset;
    L.u.a.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    L.u.a.k1 = (uint32_t)(seed >> 32);
    L.u.a.sid = stream_id;
    L.u.a.trig = trig;
    L.u.w_max = ws->w_max;
    L.u.w_max_bits = reinterpret_cast<unsigned long long*>(ws->w_max);
    L.u.counts = ws->counts;
    L.u.masks = outputs ? ws->masks : nullptr;
    L.u.values = store_values ? ws->values : nullptr;
    L.u.offsets = ws->offsets;
    L.u.range_seg = ws->range_seg;
    L.u.chunk_kept = ws->chunk_kept;
    L.u.out = p4_out_dev;
    L.u.ld = ld;
    L.u.index = index_out_dev;
    L.u.bw = inten.bw;
    for (int k = 0; k < HYDRA_PHSP_USER_PARAMS; ++k) L.u.upar[k] = inten.upar[k];
    L.max_blocks = max_blocks;
    L.pmode = pmode;
    L.intensity = inten.kind == 1 ? 1 : 0;
    void* uargs[] = {&L.u};

    const long slot = timing_begin(s);
    hipError_t e = hipSuccess;
    // the bound: given, or raised from zero to the largest trial value by the max pass
    hipLaunchKernelGGL(k_unw_set, dim3(1), dim3(64), 0, s, ws->w_max, w_max);
    e = hipGetLastError();
    if (e == hipSuccess && w_max == 0.0 && max_blocks > 0)
        e = user_max ? hipModuleLaunchKernel(user_max, (unsigned)max_blocks, 1, 1, kBlock, 1, 1, 0, s, uargs, nullptr)
                     : launch_pass_n(n_daughters, 0, L, s);
    // Chunk 0 is counted alone; then for each chunk k its scan, and its write pass
    // fused with the count of chunk k + 1 (the last chunk's write pass alone).
    auto count_range = [&](uint64_t k) {
        L.u.cnt_lo = k * chunk_segs;
        L.u.cnt_hi = std::min(segments, L.u.cnt_lo + chunk_segs);
    };
    count_range(0);
    L.blocks = ceil_div(L.u.cnt_hi - L.u.cnt_lo, (uint64_t)kUnwSegPerBlock);
    if (e == hipSuccess && L.blocks > 0)
        e = user_count ? hipModuleLaunchKernel(user_count, (unsigned)L.blocks, 1, 1, kBlock, 1, 1, 0, s, uargs, nullptr)
                       : launch_pass_n(n_daughters, 1, L, s);
    for (uint64_t k = 0; e == hipSuccess && k < nchunks; ++k) {
        const uint64_t seg_lo = k * chunk_segs, seg_hi = std::min(segments, seg_lo + chunk_segs);
        const uint64_t g_lo = seg_lo / kScanBlock, g_n = ceil_div(seg_hi - seg_lo, (uint64_t)kScanBlock);
        const bool last = k + 1 == nchunks;
        if (g_n > 0) {
            hipLaunchKernelGGL(k_unw_scan_partial, dim3((unsigned)g_n), dim3(kScanBlock), 0, s,
                               (const uint2*)ws->counts, seg_lo, seg_hi, ws->sums, ws->over_sums);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_unw_scan_top, dim3(1), dim3(kScanTop), 0, s, ws->sums + g_lo, g_n,
                               (const uint64_t*)ws->over_sums + g_lo, ws->chunk_kept, ws->chunk_over, (uint32_t)k,
                               last ? 1u : 0u, counts_dev, (const double*)ws->w_max, w_max_dev);
            e = hipGetLastError();
        }
        if (e == hipSuccess && g_n > 0 && outputs) {
            hipLaunchKernelGGL(k_unw_scan_finish, dim3((unsigned)g_n), dim3(kScanBlock), 0, s,
                               (const uint2*)ws->counts, seg_lo, seg_hi, (const uint64_t*)ws->sums, ws->offsets,
                               ws->range_seg);
            e = hipGetLastError();
        }
        if (e == hipSuccess && outputs) {
            L.u.segments = seg_hi;
            L.u.chunk = (uint32_t)k;
            L.u.last_chunk = last ? 1u : 0u;
            if (last) {
                L.write_blocks = write_blocks;
                e = launch_pass_n(n_daughters, 2, L, s);
            } else {
                count_range(k + 1);
                L.write_blocks = fused_blocks;
                e = launch_pass_n(n_daughters, 3, L, s);
            }
        }
    }
    timing_end(s, slot);
    if (e != hipSuccess) return fail_hip(e, "unweighting kernel launch");
    return HYDRA_PHSP_OK;
}

} // namespace
} // namespace hphsp

extern "C" int hydra_phsp_set_unweight_chunks(int chunks) {
    if (chunks < 0 || chunks > kMaxChunks) return fail(HYDRA_PHSP_EINVAL, "chunks must be in [0, 16]");
    g_chunks_override.store(chunks, std::memory_order_relaxed);
    return HYDRA_PHSP_OK;
}

extern "C" int hydra_phsp_generate_unweighted(double parent_mass, const double* masses_host, int n_daughters,
                                              const double* parent_p4_host, uint64_t ntrials, uint64_t seed,
                                              uint32_t stream_id, uint64_t event_offset, double w_max,
                                              double* p4_out_dev, uint64_t ld, uint64_t* index_out_dev,
                                              uint64_t* counts_dev, double* w_max_dev, void* stream) {
    MarkerRange marker("hydra_phsp_generate_unweighted");
    Channel ch;
    const int st = make_channel(parent_mass, masses_host, n_daughters, &ch);
    if (st != HYDRA_PHSP_OK) return st;
    return unweighted_run(ch, n_daughters, parent_p4_host, ntrials, seed, stream_id, event_offset, w_max, p4_out_dev,
                          ld, index_out_dev, counts_dev, w_max_dev, stream, UnwIntensity{});
}

extern "C" int hydra_phsp_generate_unweighted_model(double parent_mass, const double* masses_host, int n_daughters,
                                                    const hydra_phsp_breit_wigner* resonances_host, int n_resonances,
                                                    uint64_t ntrials, uint64_t seed, uint32_t stream_id,
                                                    uint64_t event_offset, double w_max, double* p4_out_dev,
                                                    uint64_t ld, uint64_t* index_out_dev, uint64_t* counts_dev,
                                                    double* w_max_dev, void* stream) {
    MarkerRange marker("hydra_phsp_generate_unweighted_model");
    Channel ch;
    int st = make_channel(parent_mass, masses_host, n_daughters, &ch);
    if (st != HYDRA_PHSP_OK) return st;
    UnwIntensity inten;
    st = make_bw_factors(resonances_host, n_resonances, n_daughters, &inten.bw);
    if (st != HYDRA_PHSP_OK) return st;
    // with no factor |A|^2 = 1: the weight-only passes, whose result this is
    inten.kind = inten.bw.n > 0 ? 1 : 0;
    return unweighted_run(ch, n_daughters, nullptr, ntrials, seed, stream_id, event_offset, w_max, p4_out_dev, ld,
                          index_out_dev, counts_dev, w_max_dev, stream, inten);
}

extern "C" int hydra_phsp_generate_unweighted_user_model(hydra_phsp_user_model* model, double parent_mass,
                                                         const double* masses_host, const double* params_host,
                                                         int n_params, uint64_t ntrials, uint64_t seed,
                                                         uint32_t stream_id, uint64_t event_offset, double w_max,
                                                         double* p4_out_dev, uint64_t ld, uint64_t* index_out_dev,
                                                         uint64_t* counts_dev, double* w_max_dev, void* stream) {
    MarkerRange marker("hydra_phsp_generate_unweighted_user_model");
    if (model == nullptr) return fail(HYDRA_PHSP_EINVAL, "model is NULL");
    int n = 0;
    UnwIntensity inten;
    inten.kind = 2;
    inten.user = user_model_kernels(model, &n);
    Channel ch;
    int st = make_channel(parent_mass, masses_host, n, &ch);
    if (st != HYDRA_PHSP_OK) return st;
    if (n_params < 0 || n_params > HYDRA_PHSP_USER_PARAMS)
        return fail(HYDRA_PHSP_EINVAL, "n_params must be in [0, HYDRA_PHSP_USER_PARAMS]");
    if (n_params > 0 && params_host == nullptr) return fail(HYDRA_PHSP_EINVAL, "params_host is NULL");
    for (int k = 0; k < n_params; ++k) inten.upar[k] = params_host[k];
    return unweighted_run(ch, n, nullptr, ntrials, seed, stream_id, event_offset, w_max, p4_out_dev, ld,
                          index_out_dev, counts_dev, w_max_dev, stream, inten);
}

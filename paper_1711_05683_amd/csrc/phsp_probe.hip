// phsp_probe.hip -- measurement probes: the streaming-write rate of the
// generator's output layout and the Philox call rate, each alone.
#include <hip/hip_runtime.h>

#include "hydra_phsp.h"
#include "hydra_phsp_probe.h"
#include "phsp_api_internal.hpp"
#include "phsp_kernels.hpp"

namespace hphsp {
namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeEpt = HYDRA_PHSP_PROBE_SPAN / kProbeBlock;
static_assert(kProbeEpt * kProbeBlock == HYDRA_PHSP_PROBE_SPAN, "probe span must be whole blocks");

// The generator's store sequence with constant data: block b covers
// [b * 256 * EPT, (b + 1) * 256 * EPT), lane t takes event base + k * 256 + t in
// step k, and stores every column of its event in column order, then the
// weight.  NC > 0 fixes the column count at compile time (as the generator's N
// does); NC = 0 takes it at run time.
template <int NC, int EPT>
__global__ __launch_bounds__(kProbeBlock) void k_write_bw(double* __restrict__ out, uint64_t ld, int ncols_rt,
                                                          double* __restrict__ weights, uint64_t n) {
    constexpr bool kPin = NC > 0 && NC <= 20;
    const int ncols = NC > 0 ? NC : ncols_rt;
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)(kProbeBlock * EPT);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint64_t first = base + (uint64_t)(k * kProbeBlock);
        const uint32_t off = threadIdx.x;
        if (first + off >= n) continue;
        double* o = out + first;
        const uint32_t boff = off * (uint32_t)sizeof(double);
        if constexpr (NC > 0) {
#pragma unroll
            for (int c = 0; c < NC; ++c) store_col<kPin>(o + (uint64_t)c * ld, boff, (double)c);
        } else {
            for (int c = 0; c < ncols; ++c) store_col<false>(o + (uint64_t)c * ld, boff, (double)c);
        }
        store_col<kPin>(weights + first, boff, -1.0);
    }
}

template <int NC>
hipError_t go_write(int ept, uint64_t blocks, double* out, uint64_t ld, int ncols, double* weights, uint64_t n,
                    hipStream_t s) {
    switch (ept) {
    case 1: hipLaunchKernelGGL((k_write_bw<NC, 1>), dim3((unsigned)blocks), dim3(kProbeBlock), 0, s, out, ld, ncols, weights, n); break;
    case 2: hipLaunchKernelGGL((k_write_bw<NC, 2>), dim3((unsigned)blocks), dim3(kProbeBlock), 0, s, out, ld, ncols, weights, n); break;
    case 4: hipLaunchKernelGGL((k_write_bw<NC, 4>), dim3((unsigned)blocks), dim3(kProbeBlock), 0, s, out, ld, ncols, weights, n); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Every call of the generator's Philox for the block's 1024 events, folded by
// exclusive or: lane, wave (cross-lane exchange), block (LDS).
__global__ __launch_bounds__(kProbeBlock) void k_philox_only(uint64_t n, int calls, uint32_t sid, uint32_t k0,
                                                             uint32_t k1, uint32_t* __restrict__ fold) {
    __shared__ uint32_t wave_fold[kProbeBlock / 64];
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)HYDRA_PHSP_PROBE_SPAN;
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < kProbeEpt; ++k) {
        const uint64_t e = base + (uint64_t)(k * kProbeBlock) + threadIdx.x;
        if (e < n)
            for (int j = 0; j < calls; ++j) {
                const Words4 w = philox4x32_10((uint32_t)e, (uint32_t)(e >> 32), (uint32_t)j, sid, k0, k1);
                x ^= w.x ^ w.y ^ w.z ^ w.w;
            }
    }
    for (int m = 32; m > 0; m >>= 1) x ^= (uint32_t)__shfl_xor((int)x, m, 64);
    if ((threadIdx.x & 63) == 0) wave_fold[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t b = 0;
#pragma unroll
        for (int w = 0; w < kProbeBlock / 64; ++w) b ^= wave_fold[w];
        fold[blockIdx.x] = b;
    }
}

} // namespace
} // namespace hphsp

using namespace hphsp;

extern "C" {

int hydra_phsp_probe_write(double* out_dev, uint64_t ld, int n_columns, double* weights_dev, uint64_t nevents,
                           int events_per_thread, void* stream) {
    if (out_dev == nullptr || weights_dev == nullptr) return fail(HYDRA_PHSP_EINVAL, "out_dev and weights_dev are required");
    if ((uintptr_t)out_dev % 8 || (uintptr_t)weights_dev % 8)
        return fail(HYDRA_PHSP_EINVAL, "device pointers must be 8-byte aligned");
    if (n_columns < 1 || n_columns > 4 * HYDRA_PHSP_NMAX)
        return fail(HYDRA_PHSP_EINVAL, "n_columns must be in [1, 4 * HYDRA_PHSP_NMAX]");
    if (events_per_thread != 1 && events_per_thread != 2 && events_per_thread != 4)
        return fail(HYDRA_PHSP_EINVAL, "events_per_thread must be 1, 2 or 4");
    if (ld < nevents) return fail(HYDRA_PHSP_EINVAL, "ld must be >= nevents");
    const uint64_t span = (uint64_t)kProbeBlock * (uint64_t)events_per_thread;
    const uint64_t blocks = ceil_div(nevents, span);
    if (blocks > 0xFFFFFFFFull / (uint64_t)kProbeBlock)
        return fail(HYDRA_PHSP_EINVAL, "nevents too large for one launch (more than 2^32 - 1 threads)");
    if (blocks == 0) return HYDRA_PHSP_OK;
    const hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    switch (n_columns % 4 == 0 ? n_columns / 4 : 0) {
    case 1: e = go_write<4>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    case 2: e = go_write<8>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    case 3: e = go_write<12>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    case 4: e = go_write<16>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    case 5: e = go_write<20>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    case 6: e = go_write<24>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    case 7: e = go_write<28>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    case 8: e = go_write<32>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    case 9: e = go_write<36>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    case 10: e = go_write<40>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    default: e = go_write<0>(events_per_thread, blocks, out_dev, ld, n_columns, weights_dev, nevents, s); break;
    }
    return e == hipSuccess ? HYDRA_PHSP_OK : fail_hip(e, "write probe launch");
}

int hydra_phsp_probe_philox(uint64_t nevents, int calls_per_event, uint64_t seed, uint32_t stream_id,
                            uint32_t* fold_dev, void* stream) {
    if (fold_dev == nullptr) return fail(HYDRA_PHSP_EINVAL, "fold_dev is required");
    if ((uintptr_t)fold_dev % 4) return fail(HYDRA_PHSP_EINVAL, "fold_dev must be 4-byte aligned");
    if (calls_per_event < 1 || calls_per_event > 16) return fail(HYDRA_PHSP_EINVAL, "calls_per_event must be in [1, 16]");
    const uint64_t blocks = ceil_div(nevents, HYDRA_PHSP_PROBE_SPAN);
    if (blocks > 0xFFFFFFFFull / (uint64_t)kProbeBlock)
        return fail(HYDRA_PHSP_EINVAL, "nevents too large for one launch (more than 2^32 - 1 threads)");
    if (blocks == 0) return HYDRA_PHSP_OK;
    hipLaunchKernelGGL(k_philox_only, dim3((unsigned)blocks), dim3(kProbeBlock), 0, (hipStream_t)stream, nevents,
                       calls_per_event, stream_id, (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32), fold_dev);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? HYDRA_PHSP_OK : fail_hip(e, "Philox probe launch");
}

} // extern "C"

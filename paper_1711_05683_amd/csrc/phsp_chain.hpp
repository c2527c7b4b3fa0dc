// phsp_chain.hpp -- a two-stage (sequential) decay in one launch.
//
// Sec. 4.2 of arXiv:1711.05683 lists sequential decays among the generator's
// uses: a daughter of the first decay is the parent of a second one.  The two
// single-channel calls that do it (the second with per-event parents read from
// the first one's output) are fused here: each lane computes its event of the
// first stage and stores it, keeps the chained daughter's four-momentum in
// registers, and decays it at once with the second stage's channel and counter
// stream.  The second stage's frame is built from those registers by the same
// expression the per-event-parent kernel applies to the values it reads back,
// so both stages' events and weights are bit-identical to the two calls; the
// second stage no longer reads the chained daughter's 32 bytes per event back
// from memory.  One event per lane; each stage folds its weights into its own
// block partials (merged like a single call's).
#pragma once

#include "phsp_kernels.hpp"

namespace hphsp {

template <int N1, int N2>
__global__ __launch_bounds__(kBlock) void k_phsp_chain(const KArgs a1, const KArgs a2, const int chained) {
    __shared__ double2 tab[kTrigSize];
    load_trig(tab, a1.trig);
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)kBlock;
    const uint32_t off = threadIdx.x;
    Moments acc1{0.0, 0.0, 0.0}, acc2{0.0, 0.0, 0.0};
    if (base + off < a1.nevents) {
        const uint32_t boff = off * (uint32_t)sizeof(double);
        double* const out1 = static_cast<double*>(a1.out) + base;
        double pe = 0.0, px = 0.0, py = 0.0, pz = 0.0;
        const double w1 =
            emit_event<N1, kAtRest, kFp64>(a1, base, off, tab, [&](int k, double e, double x, double y, double z) {
                store_col<(N1 <= 5)>(out1 + (uint64_t)(4 * k + 0) * a1.ld, boff, e);
                store_col<(N1 <= 5)>(out1 + (uint64_t)(4 * k + 1) * a1.ld, boff, x);
                store_col<(N1 <= 5)>(out1 + (uint64_t)(4 * k + 2) * a1.ld, boff, y);
                store_col<(N1 <= 5)>(out1 + (uint64_t)(4 * k + 3) * a1.ld, boff, z);
                if (k == chained) {
                    pe = e;
                    px = x;
                    py = y;
                    pz = z;
                }
            });
        store_col<(N1 <= 5)>(a1.weights + base, boff, w1);
        acc1 = Moments{1.0, w1, 0.0};
        const Frame f = parent_frame(pe, px, py, pz, a2.ch.M, a2.inv_M);
        double* const out2 = static_cast<double*>(a2.out) + base;
        const double w2 =
            emit_event_in_frame<N2>(a2, base, off, tab, f, [&](int k, double e, double x, double y, double z) {
                store_col<true>(out2 + (uint64_t)(4 * k + 0) * a2.ld, boff, e);
                store_col<true>(out2 + (uint64_t)(4 * k + 1) * a2.ld, boff, x);
                store_col<true>(out2 + (uint64_t)(4 * k + 2) * a2.ld, boff, y);
                store_col<true>(out2 + (uint64_t)(4 * k + 3) * a2.ld, boff, z);
            });
        store_col<true>(a2.weights + base, boff, w2);
        acc2 = Moments{1.0, w2, 0.0};
    }
    const bool full = base + (uint64_t)kBlock <= a1.nevents;
    const Moments r1 = block_reduce<kWaves>(acc1, full);
    if (threadIdx.x == 0) a1.partials[blockIdx.x] = r1;
    __syncthreads(); // the second reduction reuses the first one's LDS slots
    const Moments r2 = block_reduce<kWaves>(acc2, full);
    if (threadIdx.x == 0) a2.partials[blockIdx.x] = r2;
}

// Launcher of one first-stage daughter count (its own translation unit):
// n2 in [2, kChainN2Max], `blocks` blocks of kBlock events.
constexpr int kChainN2Max = 4;
template <int N1>
hipError_t launch_chain(int n2, const KArgs& a1, const KArgs& a2, int chained, uint64_t blocks, hipStream_t s);

} // namespace hphsp

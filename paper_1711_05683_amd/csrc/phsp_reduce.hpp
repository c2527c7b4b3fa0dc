// phsp_reduce.hpp -- integral statistics of the event weights inside a block.
#pragma once

#include <hip/hip_runtime.h>

namespace hphsp {

// Integral statistics: (n, mean, M2) with the pairwise update of Chan, Golub and
// LeVeque ("Updating formulae and a pairwise algorithm for computing sample
// variances", 1979).  Identical weights give M2 = 0 exactly.
struct Moments {
    double n, mean, m2;
};

__host__ __device__ __forceinline__ Moments merge(const Moments& a, const Moments& b) {
    if (b.n == 0.0) return a;
    if (a.n == 0.0) return b;
    const double n = a.n + b.n;
    const double delta = b.mean - a.mean;
    const double fb = b.n / n;
    Moments r;
    r.n = n;
    r.mean = a.mean + delta * fb;
    r.m2 = a.m2 + b.m2 + delta * delta * (a.n * fb);
    return r;
}

// Equal-count merge (a.n == b.n): the weights are exactly 1/2.
__device__ __forceinline__ Moments merge_equal(const Moments& a, const Moments& b) {
    const double delta = b.mean - a.mean;
    Moments r;
    r.n = a.n + b.n;
    r.mean = a.mean + delta * 0.5;
    r.m2 = a.m2 + b.m2 + delta * delta * (a.n * 0.5);
    return r;
}

__device__ __forceinline__ double shfl_down_d(double v, int off) { return __shfl_down(v, off, 64); }

// Wave-level tree (lane i absorbs lane i+off, off = 32..1); lane 0 holds the
// result.  `equal` selects the division-free form when every lane holds the
// same count.
__device__ __forceinline__ Moments wave_reduce(Moments a, bool equal) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        Moments b;
        b.n = shfl_down_d(a.n, off);
        b.mean = shfl_down_d(a.mean, off);
        b.m2 = shfl_down_d(a.m2, off);
        a = equal ? merge_equal(a, b) : merge(a, b);
    }
    return a;
}


// Block-level merge of per-lane moments; thread 0 returns the block's total.
// The cross-wave step is a pairwise tree so that equal counts stay equal.
template <int WAVES>
__device__ __forceinline__ Moments block_reduce(Moments acc, bool full) {
    __shared__ Moments sm[WAVES];
    const Moments wr = wave_reduce(acc, full);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sm[wave] = wr;
    __syncthreads();
    Moments r{0.0, 0.0, 0.0};
    if (threadIdx.x == 0) {
        Moments t[WAVES];
#pragma unroll
        for (int w = 0; w < WAVES; ++w) t[w] = sm[w];
#pragma unroll
        for (int span = 1; span < WAVES; span <<= 1)
#pragma unroll
            for (int w = 0; w + span < WAVES; w += 2 * span)
                t[w] = full ? merge_equal(t[w], t[w + span]) : merge(t[w], t[w + span]);
        r = t[0];
    }
    return r;
}

} // namespace hphsp

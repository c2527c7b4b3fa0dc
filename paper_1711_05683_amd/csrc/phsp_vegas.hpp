// phsp_vegas.hpp -- one VEGAS importance-sampling iteration on the GPU (plain
// Monte Carlo is the uniform grid).
//
// Integrand: f(x) = prod_d exp(-(x_d - mu_d)^2 / (2 s_d^2)) / (s_d sqrt(2 pi))
// over the box prod_d [lo_d, hi_d] (the paper's VEGAS benchmark integrates a
// 10-dimensional Gaussian), or a user's function of x compiled at run time.  Sample i of iteration t takes uniform d from words
// 2d, 2d+1 of the Philox stream with counter (i lo, i hi, call, t) under the
// seed; with z = K u, bin b = floor(z) and y = g[b] + (z - b)(g[b+1] - g[b]),
// x_d = lo_d + y (hi_d - lo_d), and the sample's value is f(x) times the
// Jacobian prod_d K (g[b+1] - g[b]) (hi_d - lo_d).  The iteration's estimate is
// the mean value (fused per-lane Welford, wave/LDS tree, block partials, the
// two-stage merge); the refinement histogram sums value^2 per (dimension, bin).
//
// Histogram: each wave adds into its own LDS table with LDS atomic adds; the
// block sums its four tables in wave order and writes one partial table; two
// more kernels sum the partial tables in a fixed order (groups of blocks, then
// the groups).
#pragma once

#include "phsp_device.hpp"
#include "phsp_reduce.hpp"

namespace hphsp {

constexpr int kVegasBlock = 256;
constexpr int kVegasWaves = kVegasBlock / 64;
constexpr int kVegasEpt = 4;
constexpr int kVegasDMax = 16;
constexpr int kVegasKMax = 128;

struct VegasArgs {
    int32_t bins;
    uint32_t k0, k1;             // seed
    uint32_t iteration;          // counter word 3
    uint64_t calls;
    double lo[kVegasDMax], width[kVegasDMax], mu[kVegasDMax]; // width = hi - lo
    double inv_sigma[kVegasDMax], norm[kVegasDMax];           // 1 / s_d and 1 / (s_d sqrt(2 pi)), from the host
    double upar[16];             // a user integrand's parameters (HYDRA_PHSP_USER_PARAMS of them)
    const double* grid;          // [D][bins + 1]
    Moments* partials;           // [blocks]
    double* hist_partials;       // NULL, or [blocks][D][bins]
    double* values;              // NULL, or [calls]
};

// The built-in integrand: each dimension's Gaussian factor and Jacobian are
// multiplied into the value as the dimension's coordinate is made.
// (The launch arguments come with every call rather than being held, so the
// compiler reads them where they are used, as in a plain loop.)
struct GaussIntegrand {
    double val = 1.0;
    __device__ __forceinline__ void dim(const VegasArgs& v, int d, double x, double jac) {
        const double t = (x - v.mu[d]) * v.inv_sigma[d];
        const double f = exp(-0.5 * t * t) * v.norm[d];
        val = val * f * jac;
    }
    __device__ __forceinline__ double value(const VegasArgs&) const { return val; }
};

// A VEGAS iteration with integrand type F: for every sample a block owns, a
// fresh F receives each dimension's coordinate x_d and Jacobian
// K (g[b+1] - g[b]) (hi_d - lo_d) in dimension order (dim), then gives the
// sample's value (value); the histogram and the reduction follow.  F is the
// Gaussian product above, or a user's integrand compiled at run time
// (phsp_user_model.hip).
template <int D, class F = GaussIntegrand>
__global__ __launch_bounds__(kVegasBlock) void k_vegas(const VegasArgs v) {
    extern __shared__ double vegas_lds[]; // grid [D][bins+1], then kVegasWaves tables [D][bins]
    const int K = v.bins;
    double* g = vegas_lds;
    double* tables = vegas_lds + D * (K + 1);
    const int nt = D * K;
    for (int i = threadIdx.x; i < D * (K + 1); i += kVegasBlock) g[i] = v.grid[i];
    const bool hist = v.hist_partials != nullptr;
    if (hist)
        for (int i = threadIdx.x; i < kVegasWaves * nt; i += kVegasBlock) tables[i] = 0.0;
    __syncthreads();
    double* mine = tables + (threadIdx.x >> 6) * nt;
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)(kVegasBlock * kVegasEpt);
    Moments acc{0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kVegasEpt; ++k) {
        const uint64_t i = base + (uint64_t)(k * kVegasBlock) + threadIdx.x;
        if (i < v.calls) {
            const EventRng rng{(uint32_t)i, (uint32_t)(i >> 32), v.iteration, v.k0, v.k1};
            double u[D + (D & 1)];
#pragma unroll
            for (int j = 0; 2 * j < D; ++j) rng.call((uint32_t)j, u[2 * j], u[2 * j + 1]);
            F f;
            int b[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const double z = u[d] * (double)K;
                int bb = (int)z;
                bb = bb > K - 1 ? K - 1 : bb;
                const double* gd = g + d * (K + 1);
                const double w = gd[bb + 1] - gd[bb];
                const double y = gd[bb] + (z - (double)bb) * w;
                const double x = v.lo[d] + y * v.width[d];
                f.dim(v, d, x, (double)K * w * v.width[d]);
                b[d] = bb;
            }
            const double val = f.value(v);
            if (v.values != nullptr) __builtin_nontemporal_store(val, v.values + i);
            if (hist) {
                const double v2 = val * val;
#pragma unroll
                for (int d = 0; d < D; ++d) atomicAdd(mine + d * K + b[d], v2);
            }
            if (k == 0) {
                acc = Moments{1.0, val, 0.0};
            } else {
                const double delta = val - acc.mean;
                acc.n = (double)(k + 1);
                acc.mean = acc.mean + delta * (1.0 / (double)(k + 1));
                acc.m2 = acc.m2 + delta * (val - acc.mean);
            }
        }
    }
    const bool full = base + (uint64_t)(kVegasBlock * kVegasEpt) <= v.calls;
    const Moments r = block_reduce<kVegasWaves>(acc, full); // its barrier also orders the LDS adds
    if (threadIdx.x == 0) v.partials[blockIdx.x] = r;
    if (hist) {
        double* out = v.hist_partials + (uint64_t)blockIdx.x * (uint64_t)nt;
        for (int e = threadIdx.x; e < nt; e += kVegasBlock) {
            double s = tables[e];
#pragma unroll
            for (int w = 1; w < kVegasWaves; ++w) s += tables[w * nt + e];
            out[e] = s;
        }
    }
}


struct VegasLaunch {
    VegasArgs v;
    uint64_t blocks;
    size_t lds_bytes;
};

hipError_t launch_vegas(int dim, const VegasLaunch& L, hipStream_t s);

} // namespace hphsp

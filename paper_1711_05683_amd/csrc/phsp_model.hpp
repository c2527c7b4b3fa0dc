// phsp_model.hpp -- model evaluation over phase space: every event contributes
// w |A|^2, with |A|^2 a product of relativistic Breit-Wigner intensities in pair
// invariant masses (or a user's intensity function), and the fused reduction
// integrates it.
#pragma once

#include "phsp_kernels.hpp"

namespace hphsp {

constexpr int kMaxBw = 4;
constexpr int kModelEpt = 4; // compute-bound (8 B stored per event at most)

// Breit-Wigner factors: pairs (i, j), masses and widths of the first n.
struct BwFactors {
    int32_t n;                // factors in use
    int32_t i[kMaxBw], j[kMaxBw];
    double mass[kMaxBw], width[kMaxBw];
};

struct ModelArgs {
    KArgs a;                  // channel, counters, trig table, partials (a.out unused)
    BwFactors bw;
    double* values;           // NULL or [nevents]: w |A|^2 per event
};

// The pair four-momentum p_i + p_j of an event, i and j uniform across the wave:
// every daughter is visited with compile-time indices (no dynamic register
// indexing) and added when it is i or j; adding the exact zeros of the others
// leaves the sums p_i + p_j unchanged.
template <int N>
__device__ __forceinline__ void pair_sum(const Event<N, double>& ev, int i, int j, double& e, double& x, double& y,
                                         double& z) {
    double ei = 0.0, xi = 0.0, yi = 0.0, zi = 0.0, ej = 0.0, xj = 0.0, yj = 0.0, zj = 0.0;
#pragma unroll
    for (int d = 0; d < N; ++d) {
        if (d == i) {
            ei = ev.e[d];
            xi = ev.x[d];
            yi = ev.y[d];
            zi = ev.z[d];
        }
        if (d == j) {
            ej = ev.e[d];
            xj = ev.x[d];
            yj = ev.y[d];
            zj = ev.z[d];
        }
    }
    e = ei + ej;
    x = xi + xj;
    y = yi + yj;
    z = zi + zj;
}

// |A|^2 = prod_k 1 / ((M_k^2 - s_k)^2 + (M_k G_k)^2), factors in order, with
// s = (E_i + E_j)^2 - |p_i + p_j|^2 (components summed first).
template <int N>
__device__ __forceinline__ double bw_product(const Event<N, double>& ev, const BwFactors& f) {
    double a2 = 1.0;
#pragma unroll
    for (int k = 0; k < kMaxBw; ++k) {
        if (k < f.n) {
            double e, x, y, z;
            pair_sum<N>(ev, f.i[k], f.j[k], e, x, y, z);
            const double s = e * e - x * x - y * y - z * z;
            const double d = f.mass[k] * f.mass[k] - s;
            const double mg = f.mass[k] * f.width[k];
            a2 = a2 / (d * d + mg * mg);
        }
    }
    return a2;
}

template <int N>
__device__ __forceinline__ double model_intensity(const Event<N, double>& ev, const ModelArgs& m) {
    return bw_product<N>(ev, m.bw);
}

// One block of a model kernel: every event of the block's range, with its
// weight w and its daughters' four-momenta (parent at rest), contributes
// v = w f(ev); v is stored when asked and folded into the block's partial like
// the weights of the single-channel kernel.  `f` is the intensity: the
// Breit-Wigner product below, or a user's device function compiled at run
// time (phsp_user_model.hip).
template <int N, class Intensity>
__device__ __forceinline__ void model_block(const ModelArgs& m, Intensity&& f) {
    __shared__ double2 tab[kTrigSize];
    load_trig(tab, m.a.trig);
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)(kBlock * kModelEpt);
    Moments acc{0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < kModelEpt; ++k) {
        const uint32_t off = (uint32_t)(k * kBlock) + threadIdx.x;
        if (base + off < m.a.nevents) {
            Event<N, double> ev;
            const double w = compute_event<N, kAtRest, kFp64>(m.a, base, off, tab, ev);
            const double v = w * f(ev);
            if (m.values != nullptr) __builtin_nontemporal_store(v, m.values + base + off);
            // the per-lane Welford step of the single-channel kernel
            if (k == 0) {
                acc = Moments{1.0, v, 0.0};
            } else {
                const double delta = v - acc.mean;
                acc.n = (double)(k + 1);
                acc.mean = acc.mean + delta * (1.0 / (double)(k + 1));
                acc.m2 = acc.m2 + delta * (v - acc.mean);
            }
        }
    }
    const bool full = base + (uint64_t)(kBlock * kModelEpt) <= m.a.nevents;
    const Moments r = block_reduce<kWaves>(acc, full);
    if (threadIdx.x == 0) m.a.partials[blockIdx.x] = r;
}

template <int N>
__global__ __launch_bounds__(kBlock) void k_phsp_model(const ModelArgs m) {
    model_block<N>(m, [&](const Event<N, double>& ev) { return model_intensity<N>(ev, m); });
}

template <int N>
hipError_t launch_model(const ModelArgs& m, uint64_t blocks, hipStream_t s);

} // namespace hphsp

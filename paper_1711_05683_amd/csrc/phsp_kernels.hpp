// phsp_kernels.hpp -- kernel templates of the single-channel path.
//
// k_phsp<N, PMODE, MODE, EPT>: one event per lane per step, EPT steps per lane;
// block b owns events [b*BLOCK*EPT, (b+1)*BLOCK*EPT) and in step k lane t takes
// event b*BLOCK*EPT + k*BLOCK + t, so every step's stores of one SoA column are
// BLOCK consecutive elements.  Each lane folds its weights into (n, mean, M2);
// a wave tree (shuffles), an LDS step across the block's waves and one partial
// per block follow, and a single-block finalize merges the partials in a fixed
// order (deterministic for a given launch shape).
#pragma once

#include "phsp_device.hpp"

namespace hphsp {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

enum ParentMode { kAtRest = 0, kBroadcast = 1, kPerEvent = 2 };
enum Mode { kIntegrate = 0, kFp64 = 1, kMixed = 2 };

struct KArgs {
    Channel ch;
    Frame frame;           // kBroadcast
    const double* parent;  // kPerEvent: [4][ld_parent]
    uint64_t ld_parent;
    double inv_M;          // kPerEvent
    uint64_t nevents;
    uint64_t event_offset;
    uint32_t k0, k1, sid;
    void* out;             // [N][4][ld] of double (kFp64) or float (kMixed)
    uint64_t ld;
    double* weights;       // [nevents]
    Moments* partials;     // [gridDim.x]
};

template <typename R>
__device__ __forceinline__ void store_nt(R* p, R v) {
    __builtin_nontemporal_store(v, p);
}

// Per-event parent frame: eta = P/M, gamma = E/M, 1/(gamma+1) = M/(E+M).
__device__ __forceinline__ Frame load_parent_frame(const double* parent, uint64_t ldp, uint64_t e,
                                                   double M, double inv_M) {
    const double E = parent[e];
    const double px = parent[ldp + e];
    const double py = parent[2 * ldp + e];
    const double pz = parent[3 * ldp + e];
    Frame f;
    f.eta[0] = px * inv_M;
    f.eta[1] = py * inv_M;
    f.eta[2] = pz * inv_M;
    f.gamma = E * inv_M;
    f.inv_gp1 = M / (E + M);
    return f;
}

// One event end to end: draws, levels, kinematics, lab boost, stores.
template <int N, int PMODE, int MODE>
__device__ __forceinline__ double run_event(const KArgs& a, uint64_t e) {
    Draws<N> d;
    draw_uniforms<N>(d, a.k0, a.k1, a.sid, a.event_offset + e);
    Levels<N> L;
    solve_levels<N>(a.ch, d, L);
    if constexpr (MODE != kIntegrate) {
        using R = typename std::conditional<MODE == kMixed, float, double>::type;
        Event<N, R> ev;
        build_event<N, R>(a.ch, d, L, ev);
        if constexpr (PMODE == kBroadcast) boost_to_lab<N, R>(ev, a.frame);
        if constexpr (PMODE == kPerEvent)
            boost_to_lab<N, R>(ev, load_parent_frame(a.parent, a.ld_parent, e, a.ch.M, a.inv_M));
        R* out = static_cast<R*>(a.out) + e;
        const uint64_t ld = a.ld;
#pragma unroll
        for (int k = 0; k < N; ++k) {
            store_nt(out + (uint64_t)(4 * k + 0) * ld, ev.e[k]);
            store_nt(out + (uint64_t)(4 * k + 1) * ld, ev.x[k]);
            store_nt(out + (uint64_t)(4 * k + 2) * ld, ev.y[k]);
            store_nt(out + (uint64_t)(4 * k + 3) * ld, ev.z[k]);
        }
        store_nt(a.weights + e, L.w);
    }
    return L.w;
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

template <int N, int PMODE, int MODE, int EPT>
__global__ __launch_bounds__(kBlock) void k_phsp(const KArgs a) {
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)(kBlock * EPT);
    Moments acc{0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint64_t e = base + (uint64_t)(k * kBlock) + threadIdx.x;
        if (e < a.nevents) {
            const double w = run_event<N, PMODE, MODE>(a, e);
            // Welford step with count k+1 (events of a lane form a prefix of its
            // steps).  The first event is taken as it is, so no rounding of w*w can
            // enter M2 when all weights are equal (two-body decays).
            if (k == 0) {
                acc = Moments{1.0, w, 0.0};
            } else {
                const double delta = w - acc.mean;
                acc.n = (double)(k + 1);
                acc.mean = acc.mean + delta * (1.0 / (double)(k + 1));
                acc.m2 = acc.m2 + delta * (w - acc.mean);
            }
        }
    }
    const bool full = base + (uint64_t)(kBlock * EPT) <= a.nevents;
    const Moments r = block_reduce<kWaves>(acc, full);
    if (threadIdx.x == 0) a.partials[blockIdx.x] = r;
}

// Fixed-order merge of `count` partials by one block of kFinalizeBlock threads:
// thread t folds the contiguous range [t*chunk, (t+1)*chunk) in order, then a
// wave tree and an in-order fold over the waves.
constexpr int kFinalizeBlock = 1024;

__device__ __forceinline__ void finalize_moments(const Moments* parts, uint64_t count, double* stats) {
    __shared__ Moments sm[kFinalizeBlock / 64];
    const uint64_t chunk = (count + kFinalizeBlock - 1) / kFinalizeBlock;
    const uint64_t lo = (uint64_t)threadIdx.x * chunk;
    const uint64_t hi = lo + chunk < count ? lo + chunk : count;
    Moments acc{0.0, 0.0, 0.0};
    for (uint64_t i = lo; i < hi; ++i) acc = merge(acc, parts[i]);
    const Moments wr = wave_reduce(acc, false);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = wr;
    __syncthreads();
    if (threadIdx.x == 0) {
        Moments r = sm[0];
        for (int w = 1; w < kFinalizeBlock / 64; ++w) r = merge(r, sm[w]);
        stats[0] = r.n;
        stats[1] = r.mean;
        stats[2] = r.m2;
        stats[3] = r.n >= 2.0 ? sqrt(r.m2 / ((r.n - 1.0) * r.n)) : 0.0;
    }
}

// Launch one instantiation (defined per N in its own translation unit).
struct LaunchSpec {
    int pmode;
    int mode;
    int ept;
    uint64_t blocks;
};

template <int N>
hipError_t launch_phsp(const LaunchSpec& s, const KArgs& a, hipStream_t stream);

} // namespace hphsp

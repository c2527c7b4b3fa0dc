// phsp_kernels.hpp -- kernel templates of the single-channel path.
//
// k_phsp<N, PMODE, MODE, EPT>: one event per lane per step, EPT steps per lane;
// block b owns events [b*BLOCK*EPT, (b+1)*BLOCK*EPT) and in step k lane t takes
// event b*BLOCK*EPT + k*BLOCK + t, so every step's stores of one SoA column are
// BLOCK consecutive elements.  Each lane folds its weights into (n, mean, M2);
// a wave tree (shuffles), an LDS step across the block's waves and one partial
// per block follow; the two-stage merge of the partials is in phsp_finalize.hpp.
#pragma once

#include "phsp_device.hpp"
#include "phsp_reduce.hpp"

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

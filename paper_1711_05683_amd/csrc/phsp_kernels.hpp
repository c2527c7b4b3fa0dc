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
#include "phsp_stage.hpp"

namespace hphsp {

constexpr int kBlock = 256;
static_assert(kBlock >= kTrigSize, "a block loads the trigonometric table with one entry per thread");
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
    const double2* trig;   // kTrigSize (cos, sin) pairs of 2 pi k / kTrigSize
};

// Non-temporal store to column `col` at byte offset `boff` (32-bit): the column
// base is wave-uniform, so the store takes the scalar-base + vector-offset form.
template <bool PIN, typename R>
__device__ __forceinline__ void store_col(R* col, uint32_t boff, R v) {
    if constexpr (!PIN) {
        __builtin_nontemporal_store(v, reinterpret_cast<R*>(reinterpret_cast<char*>(col) + boff));
        return;
    }
    // Pin the column base in scalar registers so the compiler does not fold the
    // columns into one per-lane 64-bit base (which costs a 64-bit add per store).
    // Only for few columns: each pinned base holds two scalar registers.
    const uint64_t p = reinterpret_cast<uint64_t>(col);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
    using gchar = __attribute__((address_space(1))) char;
    using gR = __attribute__((address_space(1))) R;
    gchar* base = (gchar*)(((uint64_t)hi << 32) | lo);
    __builtin_nontemporal_store(v, (gR*)(base + boff));
}

template <typename R>
__device__ __forceinline__ R load_col(const R* col, uint32_t boff) {
    return *reinterpret_cast<const R*>(reinterpret_cast<const char*>(col) + boff);
}

// Frame of a parent four-momentum (E, p) of mass M: eta = P/M, gamma = E/M,
// 1/(gamma+1) = M/(E+M).
__device__ __forceinline__ Frame parent_frame(double E, double px, double py, double pz, double M, double inv_M) {
    Frame f;
    f.eta[0] = px * inv_M;
    f.eta[1] = py * inv_M;
    f.eta[2] = pz * inv_M;
    f.gamma = E * inv_M;
    f.inv_gp1 = M * recip(E + M);
    return f;
}

// Per-event parent frame, read from the parent columns: `parent` already points
// at the block's first event; `off` is the lane's event offset within the block.
__device__ __forceinline__ Frame load_parent_frame(const double* parent, uint64_t ldp, uint32_t off,
                                                   double M, double inv_M) {
    const uint32_t boff = off * (uint32_t)sizeof(double);
    const double E = load_col(parent, boff);
    const double px = load_col(parent + ldp, boff);
    const double py = load_col(parent + 2 * ldp, boff);
    const double pz = load_col(parent + 3 * ldp, boff);
    return parent_frame(E, px, py, pz, M, inv_M);
}

// Counter stream of event base + off.
__device__ __forceinline__ EventRng event_rng(const KArgs& a, uint64_t base, uint32_t off) {
    const uint64_t g = a.event_offset + base + off;
    return EventRng{(uint32_t)g, (uint32_t)(g >> 32), a.sid, a.k0, a.k1};
}

// One event in the rest frame of its parent, boosted into the frame `f` moves
// with: `sink(k, e, x, y, z)` receives each daughter's final four-momentum.
template <int N, class Sink>
__device__ __forceinline__ double emit_event_in_frame(const KArgs& a, uint64_t base, uint32_t off,
                                                      const double2* tab, const Frame& f, Sink&& sink) {
    const EventRng rng = event_rng(a, base, off);
    MassDraws<N> d;
    draw_masses<N>(d, rng);
    return event_levels<N, true>(a.ch, rng, d, tab, [&](int k, double e, double x, double y, double z) {
        boost_to_lab(e, x, y, z, f);
        sink(k, e, x, y, z);
    });
}

// One event's draws, levels, kinematics and lab boost: `sink(k, e, x, y, z)`
// receives each daughter's final four-momentum (FP64) as soon as it is known
// (daughter N-1 first, 0 last; nothing for integrate-only), and the weight is
// returned.  Every kernel that needs an event goes through this, so the same
// event is bit-identical in all of them, and the mixed path's FP32 outputs are
// the FP64 outputs rounded once.
template <int N, int PMODE, int MODE, class Sink>
__device__ __forceinline__ double emit_event(const KArgs& a, uint64_t base, uint32_t off, const double2* tab,
                                             Sink&& sink) {
    if constexpr (MODE == kIntegrate || PMODE == kAtRest) {
        const EventRng rng = event_rng(a, base, off);
        MassDraws<N> d;
        draw_masses<N>(d, rng);
        return event_levels<N, MODE != kIntegrate>(a.ch, rng, d, tab, sink);
    } else {
        const Frame f = PMODE == kBroadcast ? a.frame
                                            : load_parent_frame(a.parent + base, a.ld_parent, off, a.ch.M, a.inv_M);
        return emit_event_in_frame<N>(a, base, off, tab, f, sink);
    }
}

// The same event collected in registers (for consumers that need every
// daughter at once: LDS staging, model intensities).
template <int N, int PMODE, int MODE>
__device__ __forceinline__ double compute_event(const KArgs& a, uint64_t base, uint32_t off, const double2* tab,
                                                Event<N, double>& ev) {
    return emit_event<N, PMODE, MODE>(a, base, off, tab, [&](int k, double e, double x, double y, double z) {
        ev.e[k] = e;
        ev.x[k] = x;
        ev.y[k] = y;
        ev.z[k] = z;
    });
}

// One event end to end: each daughter's four columns are stored as soon as it
// is final, then the weight.  The event is base + off: `base` (the block's first
// event) is wave-uniform, so every column address is a scalar base plus the
// lane's 32-bit offset (PIN keeps the column bases in scalar registers).  `tab`
// is the block's LDS copy of the trigonometric table.
template <int N, int PMODE, int MODE, bool PIN = (N <= 5)>
__device__ __forceinline__ double run_event(const KArgs& a, uint64_t base, uint32_t off, const double2* tab) {
    using R = typename std::conditional<MODE == kMixed, float, double>::type;
    R* const out = static_cast<R*>(a.out) + base;
    const uint64_t ld = a.ld;
    const uint32_t boff = off * (uint32_t)sizeof(R);
    const double w = emit_event<N, PMODE, MODE>(a, base, off, tab, [&](int k, double e, double x, double y, double z) {
        store_col<PIN>(out + (uint64_t)(4 * k + 0) * ld, boff, R(e));
        store_col<PIN>(out + (uint64_t)(4 * k + 1) * ld, boff, R(x));
        store_col<PIN>(out + (uint64_t)(4 * k + 2) * ld, boff, R(y));
        store_col<PIN>(out + (uint64_t)(4 * k + 3) * ld, boff, R(z));
    });
    if constexpr (MODE != kIntegrate) store_col<PIN>(a.weights + base, off * (uint32_t)sizeof(double), w);
    return w;
}

template <int N, int PMODE, int MODE, int EPT>
__global__ __launch_bounds__(kBlock) void k_phsp(const KArgs a) {
    __shared__ double2 tab[kTrigSize];
    if constexpr (MODE != kIntegrate) load_trig(tab, a.trig);
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)(kBlock * EPT);
    Moments acc{0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t off = (uint32_t)(k * kBlock) + threadIdx.x;
        if (base + off < a.nevents) {
            const double w = run_event<N, PMODE, MODE>(a, base, off, tab);
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

// k_phsp for outputs whose columns do not all start on a 128-byte line (any
// ld, any element-aligned pointer): the same events and per-lane statistics, but
// every column -- the 4N momentum columns and the weights -- is written through
// LDS in whole lines (phsp_stage.hpp), one daughter's four columns at a time.
// The body of one block of k_phsp_staged (block index blk); also a tile of the
// batched kernels.
template <int N, int PMODE, int MODE, int EPT>
__device__ __forceinline__ void run_staged_block(const KArgs& a, uint64_t blk, const double2* tab) {
    static_assert(MODE != kIntegrate, "integration stores nothing");
    static_assert(kBlock == kStageBlock, "the staging helpers assume the kernel's block size");
    using R = typename std::conditional<MODE == kMixed, float, double>::type;
    constexpr uint32_t L = line_elems<R>();
    constexpr uint32_t LW = line_elems<double>();
    __shared__ R buf[4][L + kBlock];
    __shared__ R carry[4 * N][L];
    __shared__ double wbuf[1][LW + kBlock];
    __shared__ double wcarry[1][LW];
    const uint64_t base = blk * (uint64_t)(kBlock * EPT);
    R* const out = static_cast<R*>(a.out);
    Moments acc{0.0, 0.0, 0.0};
    uint64_t next = base;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        if (next >= a.nevents) break; // uniform across the block
        const uint64_t left = a.nevents - next;
        const uint32_t total = left < (uint64_t)kBlock ? (uint32_t)left : (uint32_t)kBlock;
        const uint32_t off = (uint32_t)(k * kBlock) + threadIdx.x;
        const bool valid = threadIdx.x < total;
        Event<N, double> ev;
        double w = 0.0;
        if (valid) {
            w = compute_event<N, PMODE, MODE>(a, base, off, tab, ev);
            if (k == 0) {
                acc = Moments{1.0, w, 0.0};
            } else {
                const double delta = w - acc.mean;
                acc.n = (double)(k + 1);
                acc.mean = acc.mean + delta * (1.0 / (double)(k + 1));
                acc.m2 = acc.m2 + delta * (w - acc.mean);
            }
        }
        {
            const double wv[1] = {w};
            double* const wc[1] = {a.weights};
            const ColWindow ww[1] = {col_window<double>(line_offset(a.weights), base, next, total, a.nevents)};
            stage_and_store<1, double>(wv, valid, threadIdx.x, ww, wbuf, wcarry, wc);
        }
#pragma unroll
        for (int d = 0; d < N; ++d) {
            const R v[4] = {R(ev.e[d]), R(ev.x[d]), R(ev.y[d]), R(ev.z[d])};
            R* const cols[4] = {out + (uint64_t)(4 * d + 0) * a.ld, out + (uint64_t)(4 * d + 1) * a.ld,
                                out + (uint64_t)(4 * d + 2) * a.ld, out + (uint64_t)(4 * d + 3) * a.ld};
            ColWindow w4[4];
#pragma unroll
            for (int g = 0; g < 4; ++g) w4[g] = col_window<R>(line_offset(cols[g]), base, next, total, a.nevents);
            stage_and_store<4, R>(v, valid, threadIdx.x, w4, buf, &carry[4 * d], cols);
        }
        next += total;
    }
    flush_carry<double>(wcarry[0], a.weights, base, next, a.nevents);
    for (int c = 0; c < 4 * N; ++c) flush_carry<R>(carry[c], out + (uint64_t)c * a.ld, base, next, a.nevents);
    const bool full = base + (uint64_t)(kBlock * EPT) <= a.nevents;
    const Moments r = block_reduce<kWaves>(acc, full);
    if (threadIdx.x == 0) a.partials[blk] = r;
}

template <int N, int PMODE, int MODE, int EPT>
__global__ __launch_bounds__(kBlock) void k_phsp_staged(const KArgs a) {
    __shared__ double2 tab[kTrigSize];
    load_trig(tab, a.trig);
    run_staged_block<N, PMODE, MODE, EPT>(a, blockIdx.x, tab);
}

// Launch one instantiation (defined per N in its own translation unit).
struct LaunchSpec {
    int pmode;
    int mode;
    int ept;
    uint64_t blocks;
    bool staged; // outputs with a column off the 128-byte line grid: k_phsp_staged
};

template <int N>
hipError_t launch_phsp(const LaunchSpec& s, const KArgs& a, hipStream_t stream);

} // namespace hphsp

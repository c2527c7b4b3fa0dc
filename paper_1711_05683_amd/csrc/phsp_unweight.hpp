// phsp_unweight.hpp -- kernels of the unweighted (hit-or-miss) path.
//
// Trial event e of a launch is the weighted event the generator produces for
// the same counter; it is kept when v * w_max < w, with v the acceptance
// uniform of the event (words 0 and 1 of the first Philox call its own uniforms
// do not use).  Kept events are written in trial order.  The passes, each over
// the same blocks of kBlock * kUnwEpt trials:
//   max    (only when no bound is given) the largest weight of all trials;
//   count  kept and over-bound trials per block (weights only, no kinematics);
//   write  the full kinematics again (counter-based draws make them identical),
//          each kept event stored at its block's offset plus its rank.
// Between count and write the per-block counts are scanned (phsp_unweight_api.hip).
#pragma once

#include "phsp_kernels.hpp"
#include "phsp_stage.hpp"

namespace hphsp {

constexpr int kUnwEpt = 4; // trials per lane and block step; a block covers 1024 trials

// Philox calls of one event's own uniforms: ceil((3N - 4) / 2).
template <int N>
constexpr uint32_t kEventCalls = (uint32_t)((3 * N - 4 + 1) / 2);

template <int N>
__device__ __forceinline__ double accept_uniform(const KArgs& a, uint64_t base, uint32_t off) {
    double v, unused;
    event_rng(a, base, off).call(kEventCalls<N>, v, unused);
    return v;
}

struct UnwArgs {
    KArgs a;                   // channel, counters, parent frame, trig table (a.out unused)
    const double* w_max;       // device scalar: the bound applied
    unsigned long long* w_max_bits; // the same scalar's bits, raised by the max pass with atomic max
                                    // (non-negative doubles order like their bit patterns)
    uint2* counts;             // [blocks] (kept, weight > w_max) per block
    const uint64_t* offsets;   // [blocks] kept events before the block
    double* out;               // kept events, [N][4][ld]
    uint64_t ld;               // capacity in events
    uint64_t* index;           // NULL, or [ld] global index of each kept event
};

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Largest weight of the trials: each block's maximum raises the bound's bit
// pattern with an atomic max (exact and independent of order; the bound starts
// at zero).
template <int N>
__global__ __launch_bounds__(kBlock) void k_unw_max(const UnwArgs u) {
    __shared__ double sm[kWaves];
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)(kBlock * kUnwEpt);
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < kUnwEpt; ++k) {
        const uint32_t off = (uint32_t)(k * kBlock) + threadIdx.x;
        if (base + off < u.a.nevents) {
            Event<N, double> ev;
            m = fmax(m, compute_event<N, kAtRest, kIntegrate>(u.a, base, off, nullptr, ev));
        }
    }
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = sm[0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) r = fmax(r, sm[w]);
        // Only a block that beats the bound seen so far raises it: the bound only
        // grows, so a skipped block's maximum is already covered, and after the
        // first blocks almost none contend for the one address.
        const unsigned long long bits = (unsigned long long)__double_as_longlong(r);
        if (bits > __hip_atomic_load(u.w_max_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(u.w_max_bits, bits);
    }
}

// Kept and over-bound trials of the block (the weights only).
template <int N>
__global__ __launch_bounds__(kBlock) void k_unw_count(const UnwArgs u) {
    __shared__ uint32_t sk[kWaves], so[kWaves];
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)(kBlock * kUnwEpt);
    const double wmax = *u.w_max;
    uint32_t kept = 0, over = 0;
#pragma unroll
    for (int k = 0; k < kUnwEpt; ++k) {
        const uint32_t off = (uint32_t)(k * kBlock) + threadIdx.x;
        if (base + off < u.a.nevents) {
            Event<N, double> ev;
            const double w = compute_event<N, kAtRest, kIntegrate>(u.a, base, off, nullptr, ev);
            const double v = accept_uniform<N>(u.a, base, off);
            kept += (v * wmax < w) ? 1u : 0u;
            over += (w > wmax) ? 1u : 0u;
        }
    }
    kept = wave_sum_u32(kept);
    over = wave_sum_u32(over);
    if ((threadIdx.x & 63) == 0) {
        sk[threadIdx.x >> 6] = kept;
        so[threadIdx.x >> 6] = over;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            a += sk[w];
            b += so[w];
        }
        u.counts[blockIdx.x] = make_uint2(a, b);
    }
}

// Full kinematics of every trial, kept ones stored in trial order: step k of
// the block holds trials base + k*kBlock + t, so a kept trial's position is the
// block's offset, plus the kept trials of earlier steps, of earlier waves in
// this step, and of lower lanes in this wave.  Each column is written through
// LDS in whole 128-byte lines: a step's kept values are appended to the values
// carried over from the previous step, every completed line is stored by
// consecutive threads, and the incomplete tail is carried on; only the two lines
// at the ends of the block's run are written partially.  (Runs that start
// mid-line would otherwise turn most stores into partial-line writes.)
template <int N, int PMODE>
__global__ __launch_bounds__(kBlock) void k_unw_write(const UnwArgs u) {
    __shared__ double2 tab[kTrigSize];
    __shared__ double buf[4][line_elems<double>() + kBlock];
    __shared__ double carry[4 * N][line_elems<double>()];
    __shared__ uint64_t ibuf[1][line_elems<uint64_t>() + kBlock];
    __shared__ uint64_t icarry[1][line_elems<uint64_t>()];
    __shared__ uint32_t sk[kWaves];
    load_trig(tab, u.a.trig);
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)(kBlock * kUnwEpt);
    const double wmax = *u.w_max;
    const uint64_t first = u.offsets[blockIdx.x];
    uint64_t next = first;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < kUnwEpt; ++k) {
        const uint32_t off = (uint32_t)(k * kBlock) + threadIdx.x;
        bool keep = false;
        Event<N, double> ev;
        if (base + off < u.a.nevents) {
            const double w = compute_event<N, PMODE, kFp64>(u.a, base, off, tab, ev);
            keep = accept_uniform<N>(u.a, base, off) * wmax < w;
        }
        const uint64_t mask = __ballot(keep);
        const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                        __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        if (lane == 0) sk[wave] = (uint32_t)__popcll(mask);
        __syncthreads();
        uint32_t before = 0, total = 0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            before += (w < wave) ? sk[w] : 0u;
            total += sk[w];
        }
        const uint32_t slot = before + rank;
        if (u.index != nullptr) {
            const uint64_t g[1] = {u.a.event_offset + base + off};
            uint64_t* const icol[1] = {u.index};
            const ColWindow wi[1] = {col_window<uint64_t>(line_offset(u.index), first, next, total, u.ld)};
            stage_and_store<1, uint64_t>(g, keep, slot, wi, ibuf, icarry, icol);
        }
        if (u.out != nullptr) {
#pragma unroll
            for (int d = 0; d < N; ++d) {
                const double v[4] = {ev.e[d], ev.x[d], ev.y[d], ev.z[d]};
                double* const cols[4] = {u.out + (uint64_t)(4 * d + 0) * u.ld, u.out + (uint64_t)(4 * d + 1) * u.ld,
                                         u.out + (uint64_t)(4 * d + 2) * u.ld, u.out + (uint64_t)(4 * d + 3) * u.ld};
                ColWindow w4[4];
#pragma unroll
                for (int g = 0; g < 4; ++g) w4[g] = col_window<double>(line_offset(cols[g]), first, next, total, u.ld);
                stage_and_store<4, double>(v, keep, slot, w4, buf, &carry[4 * d], cols);
            }
        }
        next += total; // sk was read before the staging barriers, so the next step may overwrite it
    }
    if (u.index != nullptr) flush_carry<uint64_t>(icarry[0], u.index, first, next, u.ld);
    if (u.out != nullptr)
        for (int c = 0; c < 4 * N; ++c) flush_carry<double>(carry[c], u.out + (uint64_t)c * u.ld, first, next, u.ld);
}

struct UnwLaunch {
    UnwArgs u;
    uint64_t blocks;
    int pmode; // kAtRest or kBroadcast (write pass)
};

// Per-N launchers, defined in the per-N instantiation units.
template <int N>
hipError_t launch_unw_max(const UnwLaunch& L, hipStream_t s);
template <int N>
hipError_t launch_unw_count(const UnwLaunch& L, hipStream_t s);
template <int N>
hipError_t launch_unw_write(const UnwLaunch& L, hipStream_t s);

} // namespace hphsp

// phsp_unweight.hpp -- kernels of the unweighted (hit-or-miss) path.
//
// Trial event e of a launch is the weighted event the generator produces for
// the same counter; it is kept when v * w_max < w, with v the acceptance
// uniform of the event (words 0 and 1 of the first Philox call its own uniforms
// do not use).  Kept events are written in trial order.  The trials are cut
// into segments of kUnwSeg consecutive trials, one wave per segment.  The
// passes:
//   max    (only when no bound is given) the largest weight of all trials (for
//          a model, whose values cost the full kinematics, each trial's value
//          is also stored, so the count pass reads it instead of recomputing);
//   count  per segment: the keep decisions as bit masks (one 64-bit word per 64
//          trials; weights only, no kinematics), and the kept and over-bound
//          counts;
//   write  per range of kUnwRange output positions (aligned to kUnwRange, one
//          wave each): the kept trials that land in the range, listed from the
//          masks starting in the segment that holds the range's first
//          position, then the full kinematics of those trials only, lane j of
//          the wave taking output position c + j for 64-aligned c, so every
//          store covers whole lines; the kinematics are recomputed from the
//          counters (identical to the weighted events).
// Between count and write the per-segment counts are scanned and each range's
// first segment is recorded (phsp_unweight_api.hip).  The trials may be cut into
// chunks of whole scan groups: count and scan run chunk after chunk, each chunk
// carrying the kept total of the ones before it, and the write pass of a chunk
// covers the output positions its scan has settled.  A fused launch then gives
// every wave one output range of chunk k to store and one segment of chunk k+1
// to count, so the store-bound and the arithmetic-bound work share the compute
// units.  The kept set, its order and every stored value are the same for any
// chunking.
#pragma once

#include "phsp_kernels.hpp"
#include "phsp_model.hpp"

namespace hphsp {

constexpr int kUnwEpt = 4;        // max pass: trials per lane; a block covers 1024 trials
constexpr int kUnwSegWords = 16;  // mask words of a segment
constexpr int kUnwSeg = 64 * kUnwSegWords; // trials of a segment (one wave)
constexpr int kUnwSegPerBlock = kBlock / 64; // segments of a count block, ranges of a write block
constexpr int kUnwRange = 1024;   // output positions of a write-pass range (one wave)
// A range's trials are listed with 32-bit offsets from a base trial; a list is
// cut short (and the next one based anew) once its trials span this many.
constexpr uint64_t kUnwSpanLimit = 1ull << 31;

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
    uint2* counts;             // [segments] (kept, weight > w_max) per segment
    uint64_t* masks;           // NULL (count only), or [segments * kUnwSegWords] keep bits
    double* values;            // NULL, or [trials] each trial's value: stored by the max pass, read by the count
    const uint64_t* offsets;   // [segments] kept events before the segment
    const uint64_t* range_seg; // [ranges] segment holding output position r * kUnwRange
    const uint64_t* chunk_kept; // [chunks] kept trials of chunks 0..k together
    uint64_t cnt_lo, cnt_hi;   // count pass: its segments [cnt_lo, cnt_hi)
    uint64_t segments;         // write pass: segments counted so far (mask words it may read)
    uint32_t chunk;            // write pass: the chunk whose settled positions it stores
    uint32_t last_chunk;       // write pass: nonzero for the last chunk (it stores every remaining position)
    double* out;               // kept events, [N][4][ld]
    uint64_t ld;               // capacity in events
    uint64_t* index;           // NULL, or [ld] global index of each kept event
    BwFactors bw;              // a model's Breit-Wigner factors (BwIntensity)
    double upar[16];           // a user intensity's parameters (HYDRA_PHSP_USER_PARAMS of them)
};

// What a trial is accepted against: its weight w (NoIntensity), or w times a
// model's intensity of its daughters in the parent's rest frame (BwIntensity,
// or a user's function compiled at run time).  kKinematics: the intensity needs
// the daughters' four-momenta, so the trial's full event is computed.
struct NoIntensity {
    static constexpr bool kKinematics = false;
    template <int N>
    __device__ __forceinline__ double operator()(const UnwArgs&, const Event<N, double>&) const {
        return 1.0;
    }
};

struct BwIntensity {
    static constexpr bool kKinematics = true;
    template <int N>
    __device__ __forceinline__ double operator()(const UnwArgs& u, const Event<N, double>& ev) const {
        return bw_product<N>(ev, u.bw);
    }
};

// The value of trial base + off (tab: the block's trigonometric table, used only
// when the intensity needs the kinematics).
template <int N, class I>
__device__ __forceinline__ double trial_value(const UnwArgs& u, uint64_t base, uint32_t off, const double2* tab) {
    Event<N, double> ev;
    if constexpr (!I::kKinematics) {
        return compute_event<N, kAtRest, kIntegrate>(u.a, base, off, nullptr, ev);
    } else {
        const double w = compute_event<N, kAtRest, kFp64>(u.a, base, off, tab, ev);
        return w * I{}.template operator()<N>(u, ev);
    }
}

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

// Largest value of the trials: each block's maximum raises the bound's bit
// pattern with an atomic max (exact and independent of order; the bound starts
// at zero).
template <int N, class I = NoIntensity>
__global__ __launch_bounds__(kBlock) void k_unw_max(const UnwArgs u) {
    __shared__ double sm[kWaves];
    __shared__ double2 tab[I::kKinematics ? kTrigSize : 1];
    if constexpr (I::kKinematics) load_trig(tab, u.a.trig);
    const uint64_t base = (uint64_t)blockIdx.x * (uint64_t)(kBlock * kUnwEpt);
    double m = 0.0;
#pragma unroll
    for (int k = 0; k < kUnwEpt; ++k) {
        const uint32_t off = (uint32_t)(k * kBlock) + threadIdx.x;
        if (base + off < u.a.nevents) {
            const double v = trial_value<N, I>(u, base, off, tab);
            if (u.values != nullptr) u.values[base + off] = v;
            m = fmax(m, v);
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

// Keep decisions and counts of each segment (the values only: no stores).  Wave
// w of block b takes segment s = seg_lo + kUnwSegPerBlock b + w; step k covers
// its trials s kUnwSeg + 64 k + lane, and the step's ballot is the segment's
// mask word k.
template <int N, class I>
__device__ __forceinline__ void unw_count_segment(const UnwArgs& u, uint64_t seg, uint32_t lane,
                                                  const double2* tab) {
    const uint64_t base = seg * (uint64_t)kUnwSeg;
    const double wmax = *u.w_max;
    uint32_t kept = 0, over = 0;
#pragma unroll 4
    for (int k = 0; k < kUnwSegWords; ++k) {
        const uint32_t off = (uint32_t)(64 * k) + lane;
        bool keep = false, above = false;
        if (base + off < u.a.nevents) {
            const double w = u.values != nullptr ? u.values[base + off] : trial_value<N, I>(u, base, off, tab);
            const double v = accept_uniform<N>(u.a, base, off);
            keep = v * wmax < w;
            above = w > wmax;
        }
        const uint64_t m = __ballot(keep);
        kept += (uint32_t)__popcll(m);
        over += (uint32_t)__popcll(__ballot(above));
        if (u.masks != nullptr && lane == 0) u.masks[seg * kUnwSegWords + k] = m;
    }
    if (lane == 0) u.counts[seg] = make_uint2(kept, over);
}

template <int N, class I = NoIntensity>
__global__ __launch_bounds__(kBlock) void k_unw_count(const UnwArgs u) {
    __shared__ double2 tab[I::kKinematics ? kTrigSize : 1];
    if constexpr (I::kKinematics) load_trig(tab, u.a.trig); // before any wave leaves
    const uint64_t seg = u.cnt_lo + (uint64_t)blockIdx.x * kUnwSegPerBlock +
                         (uint64_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (seg < u.cnt_hi) unw_count_segment<N, I>(u, seg, threadIdx.x & 63, tab);
}

// Output positions whose trials are settled once chunks 0..k are counted and
// scanned, K the kept total of those chunks: all of them below ld when K >= ld,
// all K for the last chunk, else the whole ranges below K (the range holding K
// may still take trials of the next chunk).
__device__ __forceinline__ uint64_t unw_settled(uint64_t K, uint64_t ld, bool last) {
    if (K >= ld) return ld;
    return last ? K : K / kUnwRange * kUnwRange;
}

// Kept trials with full kinematics at their places in trial order, for the
// output positions [p0, p1) chunk k settles (p0 those settled before it, a
// multiple of kUnwRange unless it is ld).  The idx-th wave of the launch takes
// the output range r = p0 / kUnwRange + idx, positions
// [r kUnwRange, min((r + 1) kUnwRange, p1)) (list: its row of LDS).  Its first
// position lies in
// the run of segment range_seg[r]; the wave walks that segment's mask words
// and the following ones (64 words per vector load, one word per step: the
// lanes whose bit is set write their trial's offset at their rank), skipping
// the segment's kept trials before the range, until the range is full.  Then,
// for every 64-aligned window [c, c + 64) of the range, lane j computes and
// stores the event at position c + j: with columns on the 128-byte line grid
// every store covers whole lines, and no lane idles except at the very end.
// Trials are listed as 32-bit offsets from a base; should a range's trials
// spread over more than kUnwSpanLimit trials (kept fraction below about 5e-7),
// the list is stored and a new one started from the next word.
template <int N, int PMODE>
__device__ __forceinline__ void unw_write_range(const UnwArgs& u, uint64_t idx, uint32_t lane, const double2* tab,
                                                uint32_t* list) {
    const uint64_t p0 = u.chunk > 0 ? unw_settled(u.chunk_kept[u.chunk - 1], u.ld, false) : 0;
    const uint64_t stop = unw_settled(u.chunk_kept[u.chunk], u.ld, u.last_chunk != 0); // capacity truncates
    const uint64_t range = p0 / kUnwRange + idx;
    uint64_t pos = range * (uint64_t)kUnwRange;
    if (pos >= stop || p0 >= stop) return; // p0 = ld = stop: nothing left to store
    const uint64_t r1 = pos + kUnwRange < stop ? pos + kUnwRange : stop;
    const uint64_t seg = u.range_seg[range];
    uint64_t skip = pos - u.offsets[seg];                 // the segment's kept trials before the range
    uint64_t word = seg * (uint64_t)kUnwSegWords;         // next mask word to read
    const uint64_t words = u.segments * (uint64_t)kUnwSegWords;
    const bool store = u.out != nullptr;
    while (pos < r1) {
        // list the trials of positions [pos, pos + n), offsets from trial `tbase`
        const uint64_t tbase = word * 64;
        const uint32_t want = (uint32_t)(r1 - pos);
        uint32_t n = 0;
        while (n < want && word < words && word * 64 - tbase < kUnwSpanLimit) {
            const uint64_t mine = word + lane < words ? u.masks[word + lane] : 0ull;
            const uint32_t lo = (uint32_t)mine, hi = (uint32_t)(mine >> 32);
            int j = 0;
            for (; j < 64 && n < want; ++j) {
                // (readlane returns int: widen through uint32_t, not by sign extension)
                const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, j) << 32) |
                                   (uint64_t)(uint32_t)__builtin_amdgcn_readlane(lo, j);
                const uint32_t cnt = (uint32_t)__popcll(m);
                if (skip >= cnt) {
                    skip -= cnt;
                    continue;
                }
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const uint32_t at = n + rank - (uint32_t)skip; // list slot of this lane's trial
                if (((m >> lane) & 1u) && rank >= (uint32_t)skip && at < want)
                    list[at] = (uint32_t)((word + (uint64_t)j) * 64 - tbase) + lane;
                n += cnt - (uint32_t)skip;
                skip = 0;
            }
            word += (uint64_t)j;
        }
        if (n > want) n = want;
        // the list was written by other lanes of this wave: order the LDS accesses
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t c = 0; c < n; c += 64) {
            const uint32_t q = c + lane;
            if (q >= n) continue;
            const uint32_t off = list[q];
            double* const o = u.out + (pos + q);
            (void)emit_event<N, PMODE, kFp64>(u.a, tbase, off, tab,
                                              [&](int k, double e, double x, double y, double z) {
                if (store) {
                    __builtin_nontemporal_store(e, o + (uint64_t)(4 * k + 0) * u.ld);
                    __builtin_nontemporal_store(x, o + (uint64_t)(4 * k + 1) * u.ld);
                    __builtin_nontemporal_store(y, o + (uint64_t)(4 * k + 2) * u.ld);
                    __builtin_nontemporal_store(z, o + (uint64_t)(4 * k + 3) * u.ld);
                }
            });
            if (u.index != nullptr) __builtin_nontemporal_store(u.a.event_offset + tbase + off, u.index + pos + q);
        }
        pos += n;
        // the next list reuses the LDS rows only after every lane has read them
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (n == 0 && word >= words) break; // the masks ran out (not reached: the counts say so)
    }
}

template <int N, int PMODE>
__global__ __launch_bounds__(kBlock) void k_unw_write(const UnwArgs u) {
    __shared__ double2 tab[kTrigSize];
    __shared__ uint32_t list[kUnwSegPerBlock][kUnwRange];
    load_trig(tab, u.a.trig);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    unw_write_range<N, PMODE>(u, (uint64_t)blockIdx.x * kUnwSegPerBlock + wave, threadIdx.x & 63, tab, list[wave]);
}

// Fused launch: wave g counts segment u.cnt_lo + g of the next chunk, then
// stores the g-th output range chunk u.chunk settles (the two touch disjoint
// mask words: the write reads only the u.segments segments counted before).
// (Counting first also keeps the compiler from reserving a scratch slot.)
template <int N, int PMODE, class I = NoIntensity>
__global__ __launch_bounds__(kBlock) void k_unw_write_count(const UnwArgs u) {
    __shared__ double2 tab[kTrigSize];
    __shared__ uint32_t list[kUnwSegPerBlock][kUnwRange];
    load_trig(tab, u.a.trig);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t g = (uint64_t)blockIdx.x * kUnwSegPerBlock + wave;
    const uint64_t seg = u.cnt_lo + g;
    if (seg < u.cnt_hi) unw_count_segment<N, I>(u, seg, lane, tab);
    unw_write_range<N, PMODE>(u, g, lane, tab, list[wave]);
}

struct UnwLaunch {
    UnwArgs u;
    uint64_t max_blocks; // max pass: kBlock * kUnwEpt trials per block
    uint64_t blocks;     // count pass (one chunk): kUnwSegPerBlock segments per block
    uint64_t write_blocks; // write pass (one chunk): kUnwSegPerBlock ranges of kUnwRange output positions per block
                           // (fused pass: also its count segments)
    int intensity;       // max and count passes: 0 the weight alone, 1 the Breit-Wigner model (u.bw)
    int pmode;           // kAtRest or kBroadcast (write pass)
};

// Per-N launchers, defined in the per-N instantiation units.
template <int N>
hipError_t launch_unw_max(const UnwLaunch& L, hipStream_t s);
template <int N>
hipError_t launch_unw_count(const UnwLaunch& L, hipStream_t s);
template <int N>
hipError_t launch_unw_write(const UnwLaunch& L, hipStream_t s);
template <int N>
hipError_t launch_unw_write_count(const UnwLaunch& L, hipStream_t s);

} // namespace hphsp

// phsp_batch.hpp -- multi-channel (batched) kernels.
//
// Many decay channels (uneven N and event counts) run in one submission.  The
// host cuts every channel into tiles of kBlock*EPT events -- exactly the
// per-block chunks of the single-channel kernel -- groups the tiles by
// (daughter count, mode, layout) class, and per class one launch walks its tile
// range: either one block per tile, or a persistent grid with a static stride
// (block b takes tiles b, b+G, b+2G, ...; every block leaves the loop once its
// next index passes the end) or a dynamic claim of the next tile.  A class
// kernel runs the single-channel kernel's templated per-event code for its N
// (the mixed kernel of the server's ticks switches on each tile's N instead),
// and writes each tile's block partial at the channel's tile index, so events,
// weights and partials are bit-identical to a single-channel launch with the
// same events per thread; the per-channel two-stage merge then reproduces the
// single-channel integral bit for bit.
#pragma once

#include "phsp_ept.hpp"
#include "phsp_finalize.hpp"
#include "phsp_kernels.hpp"

namespace hphsp {

// One channel as the device sees it.
struct DevChannel {
    KArgs a;              // per-channel arguments (partials = channel's first tile)
    int32_t n;            // daughters
    int32_t mode;         // kFp64 or kIntegrate
    uint64_t ntiles;      // tiles (= block partials) of this channel
    uint64_t first_group; // index of the channel's first stage-1 group
    uint64_t ngroups;     // stage1_groups(ntiles)
    double* stats;        // HYDRA_PHSP_STATS doubles
};

struct TileRef {
    uint32_t channel;
    uint32_t reserved;
    uint64_t block; // block index within the channel
};

struct GroupRef {
    uint32_t channel;
    uint32_t group;
};

// The body of k_phsp for one tile, with the channel's arguments read from the
// (wave-uniform) channel record.
template <int N, int MODE, int EPT, bool PIN>
__device__ __forceinline__ void run_tile(const KArgs& a, uint64_t blk, const double2* tab) {
    const uint64_t base = blk * (uint64_t)(kBlock * EPT);
    Moments acc{0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const uint32_t off = (uint32_t)(k * kBlock) + threadIdx.x;
        if (base + off < a.nevents) {
            const double w = run_event<N, kAtRest, MODE, PIN>(a, base, off, tab);
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
    if (threadIdx.x == 0) a.partials[blk] = r;
}

// Column bases stay in scalar registers only where the kernel's scalar register
// budget allows it (every N of the kernel at most 5).
template <int N, int EPT, int NHI>
__device__ __forceinline__ void run_tile_mode(const DevChannel& c, uint64_t blk, const double2* tab) {
    constexpr bool kPin = NHI <= 5;
    if (c.mode == kIntegrate)
        run_tile<N, kIntegrate, EPT, kPin>(c.a, blk, tab);
    else
        run_tile<N, kFp64, EPT, kPin>(c.a, blk, tab);
}

// A tile of the kernel that runs every N in one launch: EPT > 0 for every
// channel, or EPT = 0 for each N and mode's single-channel default on the line
// grid (so the tile is exactly that call's block).
template <int N, int EPT, int NHI>
__device__ __forceinline__ void run_tile_any(const DevChannel& c, uint64_t blk, const double2* tab) {
    if constexpr (EPT > 0) {
        run_tile_mode<N, EPT, NHI>(c, blk, tab);
    } else {
        constexpr bool kPin = NHI <= 5;
        if (c.mode == kIntegrate)
            run_tile<N, kIntegrate, kEptIntegrate, kPin>(c.a, blk, tab);
        else
            run_tile<N, kFp64, kEptLineFp64[N], kPin>(c.a, blk, tab);
    }
}

// A value every lane of the wave holds (read from LDS), moved to scalar
// registers so that the tile and channel records are addressed uniformly.
__device__ __forceinline__ uint64_t wave_uniform(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Tile walk shared by the batched kernels.  Tiles are taken either with a
// static stride (block b: b, b+G, b+2G, ...; counter == nullptr; with G equal to
// the tile count this is one block per tile) or dynamically from a zeroed device
// counter, one atomic increment per tile, claimed while the current tile is
// being processed.  Either way every block leaves once its next index is past
// the end.  Channels of the kernel have N in [NLO, NHI]; MODE is kIntegrate or
// kFp64 for a kernel of one mode, or -1 to follow each channel's mode; STAGED
// (one N, kFp64) writes through LDS in whole lines for outputs off the line grid.
template <int NLO, int NHI, int MODE, int EPT, bool STAGED = false>
__device__ __forceinline__ void batched_body(const DevChannel* __restrict__ chans,
                                             const TileRef* __restrict__ tiles, uint64_t ntiles,
                                             const double2* __restrict__ trig,
                                             unsigned long long* __restrict__ counter) {
    __shared__ double2 tab[kTrigSize];
    __shared__ unsigned long long next;
    load_trig(tab, trig);
    const bool dynamic = counter != nullptr;
    uint64_t t = blockIdx.x;
    if (dynamic) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1ull);
        __syncthreads();
        t = wave_uniform(next);
    }
    while (t < ntiles) {
        // Thread 0 claims the block's next tile now; the claim stays in flight
        // while this tile runs and is published only after it, so the atomic's
        // round trip is hidden behind the tile.
        unsigned long long claim = 0;
        if (dynamic && threadIdx.x == 0) claim = atomicAdd(counter, 1ull);
        const TileRef tr = tiles[t];
        const DevChannel& c = chans[tr.channel];
        if constexpr (STAGED) {
            static_assert(NLO == NHI && MODE == kFp64, "staged tiles are of one N and FP64");
            run_staged_block<NLO, kAtRest, kFp64, EPT>(c.a, tr.block, tab);
        } else if constexpr (NLO == NHI && MODE >= 0) {
            run_tile<NLO, MODE, EPT, (NHI <= 5)>(c.a, tr.block, tab);
        } else {
            switch (c.n) {
            case 2: if constexpr (NLO <= 2 && NHI >= 2) run_tile_any<2, EPT, NHI>(c, tr.block, tab); break;
            case 3: if constexpr (NLO <= 3 && NHI >= 3) run_tile_any<3, EPT, NHI>(c, tr.block, tab); break;
            case 4: if constexpr (NLO <= 4 && NHI >= 4) run_tile_any<4, EPT, NHI>(c, tr.block, tab); break;
            case 5: if constexpr (NLO <= 5 && NHI >= 5) run_tile_any<5, EPT, NHI>(c, tr.block, tab); break;
            case 6: if constexpr (NLO <= 6 && NHI >= 6) run_tile_any<6, EPT, NHI>(c, tr.block, tab); break;
            case 7: if constexpr (NLO <= 7 && NHI >= 7) run_tile_any<7, EPT, NHI>(c, tr.block, tab); break;
            case 8: if constexpr (NLO <= 8 && NHI >= 8) run_tile_any<8, EPT, NHI>(c, tr.block, tab); break;
            case 9: if constexpr (NLO <= 9 && NHI >= 9) run_tile_any<9, EPT, NHI>(c, tr.block, tab); break;
            case 10: if constexpr (NLO <= 10 && NHI >= 10) run_tile_any<10, EPT, NHI>(c, tr.block, tab); break;
            default: break;
            }
        }
        if (dynamic) {
            __syncthreads(); // every wave has read `next` for this tile
            if (threadIdx.x == 0) next = claim;
        }
        // The tile's LDS reduction must finish before the next tile reuses LDS,
        // and the published claim must be visible.
        __syncthreads();
        t = dynamic ? wave_uniform(next) : t + gridDim.x;
    }
}

// Batched kernel for channels of exactly N daughters and one mode (kFp64 or
// kIntegrate), staged or not: the per-event code and the register budget are
// those of the single-channel kernel for that N, mode and layout.
template <int N, int MODE, int EPT, bool STAGED>
__global__ __launch_bounds__(kBlock)
void k_phsp_batched(const DevChannel* __restrict__ chans, const TileRef* __restrict__ tiles, uint64_t ntiles,
                    const double2* __restrict__ trig, unsigned long long* __restrict__ counter) {
    batched_body<N, N, MODE, EPT, STAGED>(chans, tiles, ntiles, trig, counter);
}

// Kernel for tiles of any N up to NMAXB in one launch (the serving path, whose
// ticks mix requests, and the batch's single-launch schedules).  EPT = 1: one
// event per thread for every N; EPT = 0: each N and mode at its single-channel
// default (kEptLineFp64, kEptIntegrate).  Its register budget is set by the
// largest N; the waves-per-SIMD hint holds it at 128 VGPRs (4 waves), which the
// top-down levels fit without spilling.
constexpr int mixed_waves_hint(int) { return 4; }

template <int NMAXB, int EPT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(mixed_waves_hint(NMAXB)))) void
k_phsp_batched_mixed(const DevChannel* __restrict__ chans, const TileRef* __restrict__ tiles, uint64_t ntiles,
                     const double2* __restrict__ trig, unsigned long long* __restrict__ counter) {
    batched_body<2, NMAXB, -1, EPT>(chans, tiles, ntiles, trig, counter);
}

// Largest grid of one launch: 256-thread blocks, at most 2^32 - 1 work-items.
constexpr uint64_t kMaxGridBlocks = 0xFFFFFFFFull / (uint64_t)kBlock;

// Zero the dynamic-schedule counters of a batch (a kernel, not a memset, so
// graph replays stay correct).
__global__ void k_zero_counters(unsigned long long* c, int n);

struct BatchLaunch {
    const DevChannel* chans;
    const TileRef* tiles;
    uint64_t ntiles;
    uint64_t grid;
    const double2* trig;
    unsigned long long* counter; // zeroed tile counter (dynamic schedule) or nullptr (static stride)
};

// Launchers, defined per instantiation unit: exactly N daughters, or any N up to
// NMAXB in one launch.
template <int N, int MODE, int EPT, bool STAGED>
hipError_t launch_batched(const BatchLaunch& b, hipStream_t stream);
template <int NMAXB, int EPT>
hipError_t launch_batched_mixed(const BatchLaunch& b, hipStream_t stream);

// Host launchers shared by the batched and serving paths: the channels of
// exactly n daughters and one mode with ept events per thread; tiles of any N
// up to nmax (8 or 10) and either mode with one event per thread (ept 1) or
// each N and mode at its single-channel default (ept 0).
hipError_t launch_batch_class(int n, int mode, bool staged, int ept, const BatchLaunch& b, hipStream_t s);
hipError_t launch_mixed_tiles(int nmax, int ept, const BatchLaunch& b, hipStream_t s);
// Stage 1 over `ngroups` group references, then stage 2 over chans[0..nch).
hipError_t launch_batch_merges(const DevChannel* chans, const GroupRef* groups, uint64_t ngroups, Moments* mid,
                               uint64_t nch, hipStream_t s);

} // namespace hphsp

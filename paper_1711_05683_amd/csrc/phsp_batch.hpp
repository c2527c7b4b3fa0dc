// phsp_batch.hpp -- persistent multi-channel kernel.
//
// Many decay channels (uneven N and event counts) run in one submission.  The
// host cuts every channel into tiles of kBlock*EPT events -- exactly the
// per-block chunks of the single-channel kernel -- groups the tiles by
// daughter-count class, and per class a persistent grid walks its tile range
// with a static stride (block b takes tiles b, b+G, b+2G, ...; every block
// leaves the loop once its next index passes the end).  Each tile switches on
// its channel's N to the same templated per-event code as the single-channel
// kernel, and writes its block partial at the channel's tile index, so events,
// weights and partials are bit-identical to a single-channel launch with the
// same events per thread; the per-channel two-stage merge then reproduces the
// single-channel integral bit for bit.
#pragma once

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

// Column bases stay in scalar registers only in the small-N classes, where the
// kernel's scalar register budget allows it.
template <int N, int EPT, int NMAXB>
__device__ __forceinline__ void run_tile_mode(const DevChannel& c, uint64_t blk, const double2* tab) {
    constexpr bool kPin = NMAXB <= 5;
    if (c.mode == kIntegrate)
        run_tile<N, kIntegrate, EPT, kPin>(c.a, blk, tab);
    else
        run_tile<N, kFp64, EPT, kPin>(c.a, blk, tab);
}

// One kernel holds the code paths of every N up to NMAXB, so its register budget
// is set by the largest; the waves-per-SIMD hint caps it (6 waves for N <= 3,
// 4 for N <= 5, 3 for N <= 8, 2 for N <= 10) instead of letting the scheduler
// trade occupancy for latency hiding.
constexpr int batch_waves_hint(int nmaxb) { return nmaxb <= 3 ? 6 : nmaxb <= 5 ? 4 : nmaxb <= 8 ? 3 : 2; }

// Tiles are taken either with a static stride (block b: b, b+G, b+2G, ...;
// counter == nullptr) or dynamically from a zeroed device counter, one atomic
// increment per tile, claimed while the previous tile is being processed, so
// blocks advance through the tile list together (as the hardware dispatcher
// would order them) and neighbouring output columns are written close in time.
// Either way every block leaves once its next index is past the end.
template <int NMAXB, int EPT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(batch_waves_hint(NMAXB)))) void k_phsp_batched(
    const DevChannel* __restrict__ chans, const TileRef* __restrict__ tiles, uint64_t ntiles,
    const double2* __restrict__ trig, unsigned long long* __restrict__ counter) {
    __shared__ double2 tab[kTrigSize];
    __shared__ unsigned long long next;
    load_trig(tab, trig);
    const bool dynamic = counter != nullptr;
    uint64_t t = blockIdx.x;
    if (dynamic) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1ull);
        __syncthreads();
        t = next;
    }
    while (t < ntiles) {
        if (dynamic) {
            __syncthreads(); // every thread holds t before `next` is overwritten
            if (threadIdx.x == 0) next = atomicAdd(counter, 1ull);
        }
        const TileRef tr = tiles[t];
        const DevChannel& c = chans[tr.channel];
        switch (c.n) {
        case 2: run_tile_mode<2, EPT, NMAXB>(c, tr.block, tab); break;
        case 3: run_tile_mode<3, EPT, NMAXB>(c, tr.block, tab); break;
        case 4: if constexpr (NMAXB >= 4) run_tile_mode<4, EPT, NMAXB>(c, tr.block, tab); break;
        case 5: if constexpr (NMAXB >= 5) run_tile_mode<5, EPT, NMAXB>(c, tr.block, tab); break;
        case 6: if constexpr (NMAXB >= 6) run_tile_mode<6, EPT, NMAXB>(c, tr.block, tab); break;
        case 7: if constexpr (NMAXB >= 7) run_tile_mode<7, EPT, NMAXB>(c, tr.block, tab); break;
        case 8: if constexpr (NMAXB >= 8) run_tile_mode<8, EPT, NMAXB>(c, tr.block, tab); break;
        case 9: if constexpr (NMAXB >= 9) run_tile_mode<9, EPT, NMAXB>(c, tr.block, tab); break;
        case 10: if constexpr (NMAXB >= 10) run_tile_mode<10, EPT, NMAXB>(c, tr.block, tab); break;
        default: break;
        }
        // The tile's LDS reduction must finish before the next tile reuses LDS,
        // and thread 0's claim of the next tile must be visible.
        __syncthreads();
        t = dynamic ? next : t + gridDim.x;
    }
}

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

// Persistent-kernel launcher for one (NMAXB, EPT) pair, defined per
// instantiation unit.
template <int NMAXB, int EPT>
hipError_t launch_batched(const BatchLaunch& b, hipStream_t stream);

// Host launchers shared by the batched and serving paths.
hipError_t launch_persistent(int nmaxb, int ept, const BatchLaunch& b, hipStream_t s);
// Stage 1 over `ngroups` group references, then stage 2 over chans[0..nch).
hipError_t launch_batch_merges(const DevChannel* chans, const GroupRef* groups, uint64_t ngroups, Moments* mid,
                               uint64_t nch, hipStream_t s);

} // namespace hphsp

// phsp_finalize.hpp -- deterministic two-stage merge of per-block moments.
//
// Stage 1: G(count) groups; group b folds the contiguous partials
// [b*per, min((b+1)*per, count)), per = ceil(count/G), with its 256 threads
// striding over the range, then a wave tree and an in-order fold of the waves.
// Stage 2: one block folds the G group results the same way and writes
// (n, mean, M2, sigma).  The tree depends only on `count`, so a channel's
// integral is bit-identical whichever launch (single-channel or batched)
// produced its partials.
#pragma once

#include "phsp_reduce.hpp"

namespace hphsp {

constexpr int kStage1Block = 256;
constexpr int kStage2Block = 1024;
constexpr uint64_t kMaxGroups = kStage2Block;
constexpr uint64_t kPartialsPerGroup = 1024;

__host__ __device__ __forceinline__ uint64_t stage1_groups(uint64_t count) {
    uint64_t g = (count + kPartialsPerGroup - 1) / kPartialsPerGroup;
    if (g < 1) g = 1;
    if (g > kMaxGroups) g = kMaxGroups;
    return g;
}

// In-order fold of per-wave results held in LDS by thread 0.
template <int WAVES>
__device__ __forceinline__ Moments fold_waves(Moments mine) {
    __shared__ Moments sm[WAVES];
    const Moments wr = wave_reduce(mine, false);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = wr;
    __syncthreads();
    Moments r{0.0, 0.0, 0.0};
    if (threadIdx.x == 0) {
        r = sm[0];
        for (int w = 1; w < WAVES; ++w) r = merge(r, sm[w]);
    }
    return r;
}

// One stage-1 group (call with kStage1Block threads).
__device__ __forceinline__ Moments stage1_group(const Moments* parts, uint64_t count, uint64_t b) {
    const uint64_t groups = stage1_groups(count);
    const uint64_t per = (count + groups - 1) / groups;
    const uint64_t lo = b * per;
    const uint64_t hi = lo + per < count ? lo + per : count;
    Moments acc{0.0, 0.0, 0.0};
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kStage1Block) acc = merge(acc, parts[i]);
    return fold_waves<kStage1Block / 64>(acc);
}

// Stage 2 (call with kStage2Block threads): fold `groups` results, write stats.
__device__ __forceinline__ void stage2_write(const Moments* mid, uint64_t groups, double* stats) {
    Moments mine{0.0, 0.0, 0.0};
    if (threadIdx.x < groups) mine = mid[threadIdx.x];
    const Moments r = fold_waves<kStage2Block / 64>(mine);
    if (threadIdx.x == 0) {
        stats[0] = r.n;
        stats[1] = r.mean;
        stats[2] = r.m2;
        stats[3] = r.n >= 2.0 ? sqrt(r.m2 / ((r.n - 1.0) * r.n)) : 0.0;
    }
}

} // namespace hphsp

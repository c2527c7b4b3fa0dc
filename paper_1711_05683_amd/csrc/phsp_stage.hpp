// phsp_stage.hpp -- line-aligned column writes through LDS.
//
// A block writes each output column as one run of consecutive positions, step
// by step (a step holds up to kBlock values).  Writing a step straight from
// registers costs partial-line writes wherever a wave's 64 values do not start
// on a 128-byte line -- for every wave when the column itself starts mid-line.
// Here a step's values are staged in LDS behind the values carried over from
// the previous step, every completed line is stored by consecutive threads, and
// the incomplete tail is carried on; only the lines at the two ends of the
// block's run are written partially (the neighbouring blocks write the rest).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hphsp {

constexpr int kStageBlock = 256; // threads of the kernels that stage (their kBlock)
constexpr uint32_t kLineBytes = 128;

template <typename T>
constexpr uint32_t line_elems() { return kLineBytes / (uint32_t)sizeof(T); }

// Window of one column for one step: positions [line0, end), end = next + total,
// line0 the start of the line holding `next`.  The first c positions are carried
// values, the first `full` complete lines (stored now), the last `tail` carried
// on.  Thread t stores window elements t and t + kStageBlock (positions pos0,
// pos0 + kStageBlock) when ok0 / ok1: within the whole lines, owned by the block
// (>= first) and below the capacity `cap`.  `mu` is the column base's element
// offset within its line.
struct ColWindow {
    uint32_t c, full, tail;
    uint64_t pos0;
    bool ok0, ok1;
};

template <typename T>
__device__ __forceinline__ uint32_t line_offset(const T* col) {
    return (uint32_t)(((uintptr_t)col / sizeof(T)) % line_elems<T>());
}

template <typename T>
__device__ __forceinline__ ColWindow col_window(uint32_t mu, uint64_t first, uint64_t next, uint32_t total,
                                                uint64_t cap) {
    constexpr uint32_t L = line_elems<T>();
    ColWindow w;
    const uint64_t line0 = next - (next + mu) % L;
    const uint64_t end = next + total;
    w.c = (uint32_t)(next - line0);
    w.full = (uint32_t)(end - (end + mu) % L - line0);
    w.tail = (uint32_t)(end - line0) - w.full;
    w.pos0 = line0 + threadIdx.x;
    const uint64_t pos1 = w.pos0 + kStageBlock;
    w.ok0 = threadIdx.x < w.full && w.pos0 >= first && w.pos0 < cap;
    w.ok1 = threadIdx.x + kStageBlock < w.full && pos1 >= first && pos1 < cap;
    return w;
}

// Stage v[g] (g < G columns; `slot` = the value's place among the step's values,
// written when `have`) behind each column's carry, store the whole lines and keep
// each tail as the new carry.  buf: G rows of line_elems + kStageBlock values;
// carry: G rows of line_elems.  Two barriers; every thread of the block calls it.
template <int G, typename T>
__device__ __forceinline__ void stage_and_store(const T (&v)[G], bool have, uint32_t slot,
                                                const ColWindow (&w)[G],
                                                T (*buf)[line_elems<T>() + kStageBlock],
                                                T (*carry)[line_elems<T>()], T* const (&col)[G]) {
    constexpr uint32_t L = line_elems<T>();
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (threadIdx.x < w[g].c) buf[g][L - w[g].c + threadIdx.x] = carry[g][threadIdx.x];
        if (have) buf[g][L + slot] = v[g];
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const uint32_t b0 = L - w[g].c + threadIdx.x;
        if (w[g].ok0) __builtin_nontemporal_store(buf[g][b0], col[g] + w[g].pos0);
        if (w[g].ok1) __builtin_nontemporal_store(buf[g][b0 + kStageBlock], col[g] + w[g].pos0 + kStageBlock);
        if (threadIdx.x < w[g].tail) carry[g][threadIdx.x] = buf[g][L - w[g].c + w[g].full + threadIdx.x];
    }
    __syncthreads(); // stores and carries have read buf before it is refilled
}

// The block's last carry of one column: the partial line at the end of its run.
template <typename T>
__device__ __forceinline__ void flush_carry(const T* carry, T* col, uint64_t first, uint64_t end, uint64_t cap) {
    constexpr uint32_t L = line_elems<T>();
    const uint64_t line0 = end - (end + line_offset(col)) % L;
    const uint64_t pos = line0 + threadIdx.x;
    if (threadIdx.x < end - line0 && pos >= first && pos < cap) __builtin_nontemporal_store(carry[threadIdx.x], col + pos);
}

} // namespace hphsp

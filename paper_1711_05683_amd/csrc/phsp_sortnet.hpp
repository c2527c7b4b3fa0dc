// phsp_sortnet.hpp -- in-register sorting networks for the N-2 mass uniforms.
//
// Size-optimal compare-exchange networks for 2..8 inputs (0, 1, 3, 5, 9, 12, 16
// and 19 comparators; Knuth, TAOCP vol. 3, sec. 5.3.4).  Each comparator (i, j),
// i < j, leaves min at i and max at j.  The tables are plain constexpr data so
// the host self-test can check them by the 0-1 principle.
#pragma once

#include <hip/hip_runtime.h>

namespace hphsp {

struct CE {
    int a, b;
};

template <int K>
struct SortNet;

template <> struct SortNet<0> { static constexpr int kSize = 0; static constexpr CE kNet[1] = {{0, 0}}; };
template <> struct SortNet<1> { static constexpr int kSize = 0; static constexpr CE kNet[1] = {{0, 0}}; };
template <> struct SortNet<2> { static constexpr int kSize = 1; static constexpr CE kNet[1] = {{0, 1}}; };
template <> struct SortNet<3> {
    static constexpr int kSize = 3;
    static constexpr CE kNet[3] = {{0, 1}, {1, 2}, {0, 1}};
};
template <> struct SortNet<4> {
    static constexpr int kSize = 5;
    static constexpr CE kNet[5] = {{0, 1}, {2, 3}, {0, 2}, {1, 3}, {1, 2}};
};
template <> struct SortNet<5> {
    static constexpr int kSize = 9;
    static constexpr CE kNet[9] = {{0, 1}, {3, 4}, {2, 4}, {2, 3}, {0, 3},
                                   {0, 2}, {1, 4}, {1, 3}, {1, 2}};
};
template <> struct SortNet<6> {
    static constexpr int kSize = 12;
    static constexpr CE kNet[12] = {{1, 2}, {4, 5}, {0, 2}, {3, 5}, {0, 1}, {3, 4},
                                    {2, 5}, {0, 3}, {1, 4}, {2, 4}, {1, 3}, {2, 3}};
};
template <> struct SortNet<7> {
    static constexpr int kSize = 16;
    static constexpr CE kNet[16] = {{1, 2}, {3, 4}, {5, 6}, {0, 2}, {3, 5}, {4, 6}, {0, 1}, {4, 5},
                                    {2, 6}, {0, 4}, {1, 5}, {0, 3}, {2, 5}, {1, 3}, {2, 4}, {2, 3}};
};
template <> struct SortNet<8> {
    static constexpr int kSize = 19;
    static constexpr CE kNet[19] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6},
                                    {3, 7}, {0, 1}, {2, 3}, {4, 5}, {6, 7}, {2, 4}, {3, 5},
                                    {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
};

// Compare-exchange primitives: min/max instructions for doubles (inputs are
// never NaN), plain comparisons for the host self-test's integers.
__host__ __device__ __forceinline__ double ce_lo(double a, double b) { return fmin(a, b); }
__host__ __device__ __forceinline__ double ce_hi(double a, double b) { return fmax(a, b); }
__host__ __device__ __forceinline__ int ce_lo(int a, int b) { return a < b ? a : b; }
__host__ __device__ __forceinline__ int ce_hi(int a, int b) { return a < b ? b : a; }

// Sort v[0..K-1] ascending in registers (NaN-free inputs).
template <int K, typename T>
__host__ __device__ __forceinline__ void sortnet_sort(T* v) {
#pragma unroll
    for (int c = 0; c < SortNet<K>::kSize; ++c) {
        const int a = SortNet<K>::kNet[c].a, b = SortNet<K>::kNet[c].b;
        const T lo = ce_lo(v[a], v[b]);
        const T hi = ce_hi(v[a], v[b]);
        v[a] = lo;
        v[b] = hi;
    }
}

} // namespace hphsp

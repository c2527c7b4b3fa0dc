// phsp_batch_inst.hip -- instantiates the batched kernels of one unit: compiled
// once per N with -DBATCH_N=<2..10> (exact-N kernels: FP64 direct and staged,
// integrate-only; 1, 2 and 4 events per thread) and once per bound with -DBATCH_MIXED=<8|10> (any N up to the bound,
// one event per thread, or each N at its single-channel default).
#include "phsp_batch.hpp"

#if !defined(BATCH_N) && !defined(BATCH_MIXED)
#error "compile with -DBATCH_N=<2..10> or -DBATCH_MIXED=<8|10>"
#endif

namespace hphsp {

#if defined(BATCH_N)
template <int MODE, int EPT, bool STAGED>
static hipError_t launch_n(const BatchLaunch& b, hipStream_t stream) {
    if (b.grid == 0 || b.grid > kMaxGridBlocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_phsp_batched<BATCH_N, MODE, EPT, STAGED>), dim3((unsigned)b.grid), dim3(kBlock), 0,
                       stream, b.chans, b.tiles, b.ntiles, b.trig, b.counter);
    return hipGetLastError();
}
#define HPHSP_BATCH_INST(MODE, EPT, STAGED)                                                                    \
    template <>                                                                                                \
    hipError_t launch_batched<BATCH_N, MODE, EPT, STAGED>(const BatchLaunch& b, hipStream_t s) {              \
        return launch_n<MODE, EPT, STAGED>(b, s);                                                              \
    }
HPHSP_BATCH_INST(kFp64, 1, false)
HPHSP_BATCH_INST(kFp64, 2, false)
HPHSP_BATCH_INST(kFp64, 4, false)
HPHSP_BATCH_INST(kFp64, 1, true)
HPHSP_BATCH_INST(kFp64, 2, true)
HPHSP_BATCH_INST(kFp64, 4, true)
HPHSP_BATCH_INST(kIntegrate, 1, false)
HPHSP_BATCH_INST(kIntegrate, 2, false)
HPHSP_BATCH_INST(kIntegrate, 4, false)
#undef HPHSP_BATCH_INST
#endif

#if defined(BATCH_MIXED)
template <int EPT>
static hipError_t launch_mixed(const BatchLaunch& b, hipStream_t stream) {
    if (b.grid == 0 || b.grid > kMaxGridBlocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_phsp_batched_mixed<BATCH_MIXED, EPT>), dim3((unsigned)b.grid), dim3(kBlock), 0, stream,
                       b.chans, b.tiles, b.ntiles, b.trig, b.counter);
    return hipGetLastError();
}
template <>
hipError_t launch_batched_mixed<BATCH_MIXED, 1>(const BatchLaunch& b, hipStream_t stream) {
    return launch_mixed<1>(b, stream);
}
template <>
hipError_t launch_batched_mixed<BATCH_MIXED, 0>(const BatchLaunch& b, hipStream_t stream) {
    return launch_mixed<0>(b, stream);
}
#endif

} // namespace hphsp

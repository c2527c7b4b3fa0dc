// phsp_batch_inst.hip -- instantiates the persistent multi-channel kernel for one
// (largest N, events per thread) pair; compiled once per pair with
// -DBATCH_NMAX=<8|10> -DBATCH_EPT=<1|2|4>.
#include "phsp_batch.hpp"

#if !defined(BATCH_NMAX) || !defined(BATCH_EPT)
#error "compile with -DBATCH_NMAX=<8|10> -DBATCH_EPT=<1|2|4>"
#endif

namespace hphsp {

template <>
hipError_t launch_batched<BATCH_NMAX, BATCH_EPT>(const BatchLaunch& b, hipStream_t stream) {
    if (b.grid == 0 || b.grid > 0x7FFFFFFFull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_phsp_batched<BATCH_NMAX, BATCH_EPT>), dim3((unsigned)b.grid), dim3(kBlock), 0,
                       stream, b.chans, b.tiles, b.ntiles, b.trig, b.counter);
    return hipGetLastError();
}

} // namespace hphsp

// phsp_model_inst.hip -- instantiates the model-evaluation kernel for one
// daughter count; compiled once per N with -DMODEL_N=<2..10>.
#include "phsp_model.hpp"

#ifndef MODEL_N
#error "compile with -DMODEL_N=<2..10>"
#endif

namespace hphsp {

template <>
hipError_t launch_model<MODEL_N>(const ModelArgs& m, uint64_t blocks, hipStream_t s) {
    if (blocks == 0 || blocks > 0xFFFFFFFFull / (uint64_t)kBlock) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_phsp_model<MODEL_N>), dim3((unsigned)blocks), dim3(kBlock), 0, s, m);
    return hipGetLastError();
}

} // namespace hphsp

// phsp_chain_inst.hip -- instantiates the two-stage kernel for one first-stage
// daughter count and every second-stage count; compiled once per N1 with
// -DCHAIN_N1=<2..10>.
#include "phsp_chain.hpp"

#ifndef CHAIN_N1
#error "compile with -DCHAIN_N1=<2..10>"
#endif

namespace hphsp {

template <>
hipError_t launch_chain<CHAIN_N1>(int n2, const KArgs& a1, const KArgs& a2, int chained, uint64_t blocks,
                                  hipStream_t s) {
    if (blocks == 0 || blocks > 0xFFFFFFFFull / (uint64_t)kBlock || chained < 0 || chained >= CHAIN_N1)
        return hipErrorInvalidValue;
    static_assert(kChainN2Max == 4, "one case per second-stage daughter count");
    switch (n2) {
    case 2: hipLaunchKernelGGL((k_phsp_chain<CHAIN_N1, 2>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a1, a2, chained); break;
    case 3: hipLaunchKernelGGL((k_phsp_chain<CHAIN_N1, 3>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a1, a2, chained); break;
    case 4: hipLaunchKernelGGL((k_phsp_chain<CHAIN_N1, 4>), dim3((unsigned)blocks), dim3(kBlock), 0, s, a1, a2, chained); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace hphsp

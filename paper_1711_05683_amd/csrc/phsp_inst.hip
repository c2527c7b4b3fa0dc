// phsp_inst.hip -- instantiates the single-channel kernels for one daughter
// count.  Compiled once per N (2..10) with -DPHSP_N=<N>, so the instantiations
// build in parallel.
#include "phsp_kernels.hpp"

#ifndef PHSP_N
#error "compile with -DPHSP_N=<number of daughters>"
#endif

namespace hphsp {

namespace {

template <int PMODE, int MODE, int EPT>
hipError_t go(const LaunchSpec& s, const KArgs& a, hipStream_t stream) {
    if constexpr (MODE != kIntegrate) {
        if (s.staged) {
            hipLaunchKernelGGL((k_phsp_staged<PHSP_N, PMODE, MODE, EPT>), dim3((unsigned)s.blocks), dim3(kBlock), 0,
                               stream, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_phsp<PHSP_N, PMODE, MODE, EPT>), dim3((unsigned)s.blocks), dim3(kBlock), 0,
                       stream, a);
    return hipGetLastError();
}

template <int PMODE, int MODE>
hipError_t by_ept(const LaunchSpec& s, const KArgs& a, hipStream_t stream) {
    switch (s.ept) {
    case 1: return go<PMODE, MODE, 1>(s, a, stream);
    case 2: return go<PMODE, MODE, 2>(s, a, stream);
    case 4: return go<PMODE, MODE, 4>(s, a, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int PMODE>
hipError_t by_mode(const LaunchSpec& s, const KArgs& a, hipStream_t stream) {
    switch (s.mode) {
    case kFp64: return by_ept<PMODE, kFp64>(s, a, stream);
    case kMixed: return by_ept<PMODE, kMixed>(s, a, stream);
    default: return hipErrorInvalidValue;
    }
}

} // namespace

template <>
hipError_t launch_phsp<PHSP_N>(const LaunchSpec& s, const KArgs& a, hipStream_t stream) {
    if (s.blocks == 0 || s.blocks > 0xFFFFFFFFull / (uint64_t)kBlock) return hipErrorInvalidValue;
    if (s.mode == kIntegrate) return by_ept<kAtRest, kIntegrate>(s, a, stream);
    switch (s.pmode) {
    case kAtRest: return by_mode<kAtRest>(s, a, stream);
    case kBroadcast: return by_mode<kBroadcast>(s, a, stream);
    case kPerEvent: return by_mode<kPerEvent>(s, a, stream);
    default: return hipErrorInvalidValue;
    }
}

} // namespace hphsp

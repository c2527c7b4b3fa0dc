// phsp_unweight_inst.hip -- instantiates the unweighted-path kernels for one
// daughter count; compiled once per N with -DUNW_N=<2..10>.
#include "phsp_unweight.hpp"

#ifndef UNW_N
#error "compile with -DUNW_N=<2..10>"
#endif

namespace hphsp {

static bool grid_ok(uint64_t blocks) { return blocks > 0 && blocks <= 0xFFFFFFFFull / (uint64_t)kBlock; }

template <>
hipError_t launch_unw_max<UNW_N>(const UnwLaunch& L, hipStream_t s) {
    if (!grid_ok(L.max_blocks)) return hipErrorInvalidValue;
    if (L.intensity == 1)
        hipLaunchKernelGGL((k_unw_max<UNW_N, BwIntensity>), dim3((unsigned)L.max_blocks), dim3(kBlock), 0, s, L.u);
    else
        hipLaunchKernelGGL((k_unw_max<UNW_N>), dim3((unsigned)L.max_blocks), dim3(kBlock), 0, s, L.u);
    return hipGetLastError();
}

template <>
hipError_t launch_unw_count<UNW_N>(const UnwLaunch& L, hipStream_t s) {
    if (!grid_ok(L.blocks)) return hipErrorInvalidValue;
    if (L.intensity == 1)
        hipLaunchKernelGGL((k_unw_count<UNW_N, BwIntensity>), dim3((unsigned)L.blocks), dim3(kBlock), 0, s, L.u);
    else
        hipLaunchKernelGGL((k_unw_count<UNW_N>), dim3((unsigned)L.blocks), dim3(kBlock), 0, s, L.u);
    return hipGetLastError();
}

template <>
hipError_t launch_unw_write<UNW_N>(const UnwLaunch& L, hipStream_t s) {
    if (!grid_ok(L.write_blocks) || L.u.masks == nullptr) return hipErrorInvalidValue;
    if (L.pmode == kBroadcast)
        hipLaunchKernelGGL((k_unw_write<UNW_N, kBroadcast>), dim3((unsigned)L.write_blocks), dim3(kBlock), 0, s, L.u);
    else
        hipLaunchKernelGGL((k_unw_write<UNW_N, kAtRest>), dim3((unsigned)L.write_blocks), dim3(kBlock), 0, s, L.u);
    return hipGetLastError();
}

template <>
hipError_t launch_unw_write_count<UNW_N>(const UnwLaunch& L, hipStream_t s) {
    if (!grid_ok(L.write_blocks) || L.u.masks == nullptr) return hipErrorInvalidValue;
    if (L.intensity == 1)
        hipLaunchKernelGGL((k_unw_write_count<UNW_N, kAtRest, BwIntensity>), dim3((unsigned)L.write_blocks),
                           dim3(kBlock), 0, s, L.u);
    else if (L.pmode == kBroadcast)
        hipLaunchKernelGGL((k_unw_write_count<UNW_N, kBroadcast>), dim3((unsigned)L.write_blocks), dim3(kBlock), 0,
                           s, L.u);
    else
        hipLaunchKernelGGL((k_unw_write_count<UNW_N, kAtRest>), dim3((unsigned)L.write_blocks), dim3(kBlock), 0, s,
                           L.u);
    return hipGetLastError();
}

} // namespace hphsp

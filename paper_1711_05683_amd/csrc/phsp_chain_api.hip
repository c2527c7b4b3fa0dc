// phsp_chain_api.hip -- C ABI of the two-stage decay in one launch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "hydra_phsp.h"
#include "phsp_api_internal.hpp"
#include "phsp_chain.hpp"

namespace hphsp {
namespace {

hipError_t launch_chain_n(int n1, int n2, const KArgs& a1, const KArgs& a2, int chained, uint64_t blocks,
                          hipStream_t s) {
    switch (n1) {
    case 2: return launch_chain<2>(n2, a1, a2, chained, blocks, s);
    case 3: return launch_chain<3>(n2, a1, a2, chained, blocks, s);
    case 4: return launch_chain<4>(n2, a1, a2, chained, blocks, s);
    case 5: return launch_chain<5>(n2, a1, a2, chained, blocks, s);
    case 6: return launch_chain<6>(n2, a1, a2, chained, blocks, s);
    case 7: return launch_chain<7>(n2, a1, a2, chained, blocks, s);
    case 8: return launch_chain<8>(n2, a1, a2, chained, blocks, s);
    case 9: return launch_chain<9>(n2, a1, a2, chained, blocks, s);
    case 10: return launch_chain<10>(n2, a1, a2, chained, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

bool on_line_grid(const void* p, uint64_t ld_bytes) {
    return (uintptr_t)p % kLineBytes == 0 && ld_bytes % kLineBytes == 0;
}

} // namespace
} // namespace hphsp

using namespace hphsp;

extern "C" int hydra_phsp_generate_chain(double parent_mass, const double* masses_host, int n_daughters,
                                         int chained, const double* masses2_host, int n2, uint64_t nevents,
                                         uint64_t seed, uint32_t stream_id, uint32_t stream_id2,
                                         uint64_t event_offset, double* p4_out_dev, uint64_t ld,
                                         double* weights_dev, double* stats_dev, double* p4_out2_dev,
                                         uint64_t ld2, double* weights2_dev, double* stats2_dev, void* stream) {
    MarkerRange marker("hydra_phsp_generate_chain");
    Channel c1, c2;
    int st = make_channel(parent_mass, masses_host, n_daughters, &c1);
    if (st != HYDRA_PHSP_OK) return st;
    if (chained < 0 || chained >= n_daughters)
        return fail(HYDRA_PHSP_EINVAL, "chained must name a daughter of the first stage");
    if (n2 < 2 || n2 > kChainN2Max) return fail(HYDRA_PHSP_EINVAL, "n2 must be in [2, 4]");
    st = make_channel(masses_host[chained], masses2_host, n2, &c2);
    if (st != HYDRA_PHSP_OK) return st;
    if (nevents > 0 && (p4_out_dev == nullptr || weights_dev == nullptr || p4_out2_dev == nullptr ||
                        weights2_dev == nullptr))
        return fail(HYDRA_PHSP_EINVAL, "both stages' p4 and weight outputs are required");
    if (ld < nevents || ld2 < nevents) return fail(HYDRA_PHSP_EINVAL, "ld and ld2 must be >= nevents");
    const void* ptrs[6] = {p4_out_dev, weights_dev, stats_dev, p4_out2_dev, weights2_dev, stats2_dev};
    for (const void* p : ptrs)
        if ((uintptr_t)p % sizeof(double) != 0)
            return fail(HYDRA_PHSP_EINVAL, "device pointers must be aligned to their element size");
    const uint64_t blocks = ceil_div(nevents, (uint64_t)kBlock);
    if (blocks > 0xFFFFFFFFull / (uint64_t)kBlock)
        return fail(HYDRA_PHSP_EINVAL, "nevents too large for one launch (more than 2^32 - 1 threads)");
    hipStream_t s = (hipStream_t)stream;
    // Columns off the 128-byte line grid: the two single-channel calls, whose
    // staged kernels write whole lines (the fused kernel stores directly).
    const bool fused = on_line_grid(p4_out_dev, ld * sizeof(double)) && on_line_grid(weights_dev, 0) &&
                       on_line_grid(p4_out2_dev, ld2 * sizeof(double)) && on_line_grid(weights2_dev, 0);
    if (!fused) {
        st = run_single(c1, n_daughters, kAtRest, nullptr, nullptr, 0, nevents, seed, stream_id, event_offset,
                        kFp64, p4_out_dev, ld, weights_dev, stats_dev, s, 0);
        if (st != HYDRA_PHSP_OK) return st;
        return run_single(c2, n2, kPerEvent, nullptr, p4_out_dev + (uint64_t)(4 * chained) * ld, ld, nevents,
                          seed, stream_id2, event_offset, kFp64, p4_out2_dev, ld2, weights2_dev, stats2_dev, s, 0);
    }
    Moments* partials = nullptr;
    st = block_partials(s, 2 * std::max<uint64_t>(blocks, 1), &partials);
    if (st != HYDRA_PHSP_OK) return st;
    const double2* trig = nullptr;
    st = trig_table(&trig);
    if (st != HYDRA_PHSP_OK) return st;
    KArgs a1, a2;
    std::memset(&a1, 0, sizeof(a1));
    std::memset(&a2, 0, sizeof(a2));
    a1.ch = c1;
    a1.inv_M = 1.0 / c1.M;
    a1.nevents = nevents;
    a1.event_offset = event_offset;
    a1.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    a1.k1 = (uint32_t)(seed >> 32);
    a1.sid = stream_id;
    a1.out = p4_out_dev;
    a1.ld = ld;
    a1.weights = weights_dev;
    a1.partials = partials;
    a1.trig = trig;
    a2 = a1;
    a2.ch = c2;
    a2.inv_M = 1.0 / c2.M;
    a2.sid = stream_id2;
    a2.out = p4_out2_dev;
    a2.ld = ld2;
    a2.weights = weights2_dev;
    a2.partials = partials + blocks;
    if (blocks > 0) {
        const long slot = timing_begin(s);
        const hipError_t e = launch_chain_n(n_daughters, n2, a1, a2, chained, blocks, s);
        timing_end(s, slot);
        if (e != hipSuccess) return fail_hip(e, "two-stage kernel launch");
    }
    if (stats_dev != nullptr) {
        st = merge_partials(s, a1.partials, blocks, stats_dev);
        if (st != HYDRA_PHSP_OK) return st;
    }
    if (stats2_dev != nullptr) return merge_partials(s, a2.partials, blocks, stats2_dev);
    return HYDRA_PHSP_OK;
}

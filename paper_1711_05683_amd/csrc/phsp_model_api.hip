// phsp_model_api.hip -- C ABI of model evaluation over phase space.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "hydra_phsp.h"
#include "hydra_phsp_model.h"
#include "phsp_api_internal.hpp"
#include "phsp_model.hpp"

namespace hphsp {

int make_bw_factors(const hydra_phsp_breit_wigner* res, int n_res, int n_daughters, BwFactors* out) {
    std::memset(out, 0, sizeof(*out));
    if (n_res < 0 || n_res > HYDRA_PHSP_MAX_BW)
        return fail(HYDRA_PHSP_EINVAL, "n_resonances must be in [0, HYDRA_PHSP_MAX_BW]");
    if (n_res > 0 && res == nullptr) return fail(HYDRA_PHSP_EINVAL, "resonances_host is NULL");
    out->n = n_res;
    for (int k = 0; k < n_res; ++k) {
        const hydra_phsp_breit_wigner& r = res[k];
        if (r.i < 0 || r.j >= n_daughters || r.i >= r.j)
            return fail(HYDRA_PHSP_EINVAL, "resonance pair must satisfy 0 <= i < j < n_daughters");
        if (!(r.mass > 0.0) || !(r.width > 0.0) || !std::isfinite(r.mass) || !std::isfinite(r.width))
            return fail(HYDRA_PHSP_EINVAL, "resonance mass and width must be finite and > 0");
        out->i[k] = r.i;
        out->j[k] = r.j;
        out->mass[k] = r.mass;
        out->width[k] = r.width;
    }
    return HYDRA_PHSP_OK;
}

namespace {

hipError_t launch_model_n(int n, const ModelArgs& m, uint64_t blocks, hipStream_t s) {
    switch (n) {
    case 2: return launch_model<2>(m, blocks, s);
    case 3: return launch_model<3>(m, blocks, s);
    case 4: return launch_model<4>(m, blocks, s);
    case 5: return launch_model<5>(m, blocks, s);
    case 6: return launch_model<6>(m, blocks, s);
    case 7: return launch_model<7>(m, blocks, s);
    case 8: return launch_model<8>(m, blocks, s);
    case 9: return launch_model<9>(m, blocks, s);
    case 10: return launch_model<10>(m, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

} // namespace
} // namespace hphsp

using namespace hphsp;

extern "C" int hydra_phsp_integrate_model(double parent_mass, const double* masses_host, int n_daughters,
                                          const hydra_phsp_breit_wigner* resonances_host, int n_resonances,
                                          uint64_t nevents, uint64_t seed, uint32_t stream_id,
                                          uint64_t event_offset, double* values_dev, double* stats_dev,
                                          void* stream) {
    MarkerRange marker("hydra_phsp_integrate_model");
    Channel ch;
    int st = make_channel(parent_mass, masses_host, n_daughters, &ch);
    if (st != HYDRA_PHSP_OK) return st;
    if (stats_dev == nullptr) return fail(HYDRA_PHSP_EINVAL, "stats_dev is required");
    if ((uintptr_t)values_dev % sizeof(double) != 0 || (uintptr_t)stats_dev % sizeof(double) != 0)
        return fail(HYDRA_PHSP_EINVAL, "device pointers must be aligned to their element size");
    ModelArgs m;
    std::memset(&m, 0, sizeof(m));
    st = make_bw_factors(resonances_host, n_resonances, n_daughters, &m.bw);
    if (st != HYDRA_PHSP_OK) return st;
    const uint64_t span = (uint64_t)kBlock * (uint64_t)kModelEpt;
    const uint64_t blocks = ceil_div(nevents, span);
    if (blocks > 0xFFFFFFFFull / (uint64_t)kBlock)
        return fail(HYDRA_PHSP_EINVAL, "nevents too large for one launch (more than 2^32 - 1 threads)");
    hipStream_t s = (hipStream_t)stream;
    Moments* partials = nullptr;
    st = block_partials(s, blocks, &partials);
    if (st != HYDRA_PHSP_OK) return st;
    const double2* trig = nullptr;
    st = trig_table(&trig);
    if (st != HYDRA_PHSP_OK) return st;
    m.a.ch = ch;
    m.a.inv_M = 1.0 / ch.M;
    m.a.nevents = nevents;
    m.a.event_offset = event_offset;
    m.a.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    m.a.k1 = (uint32_t)(seed >> 32);
    m.a.sid = stream_id;
    m.a.partials = partials;
    m.a.trig = trig;
    m.values = values_dev;
    if (blocks > 0) {
        const long slot = timing_begin(s);
        const hipError_t e = launch_model_n(n_daughters, m, blocks, s);
        timing_end(s, slot);
        if (e != hipSuccess) return fail_hip(e, "model kernel launch");
    }
    return merge_partials(s, partials, blocks, stats_dev);
}

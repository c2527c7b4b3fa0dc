// phsp_vegas_api.hip -- VEGAS / plain Monte Carlo: kernel instantiations, the
// host-side grid refinement and the C ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "hydra_phsp.h"
#include "hydra_phsp_vegas.h"
#include "phsp_api_internal.hpp"
#include "phsp_vegas.hpp"

namespace hphsp {

static_assert(sizeof(VegasArgs::upar) / sizeof(double) == HYDRA_PHSP_USER_PARAMS,
              "a user integrand's parameters travel in VegasArgs::upar");

// Histogram sum over the per-block tables in two fixed-order stages: group g
// (blockIdx.y) sums the tables of blocks [g * kHistGroup, (g + 1) * kHistGroup)
// entry by entry, then one pass sums the group results in group order.
constexpr uint64_t kHistGroup = 256;

__global__ __launch_bounds__(256) void k_vegas_hist_groups(const double* __restrict__ partials, uint64_t blocks,
                                                           int entries, double* __restrict__ mid) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= entries) return;
    const uint64_t b0 = (uint64_t)blockIdx.y * kHistGroup;
    const uint64_t b1 = b0 + kHistGroup < blocks ? b0 + kHistGroup : blocks;
    double s = 0.0;
    for (uint64_t b = b0; b < b1; ++b) s += partials[b * (uint64_t)entries + e];
    mid[(uint64_t)blockIdx.y * (uint64_t)entries + e] = s;
}

__global__ __launch_bounds__(256) void k_vegas_hist_sum(const double* __restrict__ mid, uint64_t groups,
                                                        int entries, double* __restrict__ hist) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= entries) return;
    double s = 0.0;
    for (uint64_t g = 0; g < groups; ++g) s += mid[g * (uint64_t)entries + e];
    hist[e] = s;
}

template <int D>
static hipError_t go(const VegasLaunch& L, hipStream_t s) {
    hipLaunchKernelGGL((k_vegas<D>), dim3((unsigned)L.blocks), dim3(kVegasBlock), L.lds_bytes, s, L.v);
    return hipGetLastError();
}

hipError_t launch_vegas(int dim, const VegasLaunch& L, hipStream_t s) {
    if (L.blocks == 0 || L.blocks > 0xFFFFFFFFull / (uint64_t)kVegasBlock) return hipErrorInvalidValue;
    switch (dim) {
    case 1: return go<1>(L, s);
    case 2: return go<2>(L, s);
    case 3: return go<3>(L, s);
    case 4: return go<4>(L, s);
    case 5: return go<5>(L, s);
    case 6: return go<6>(L, s);
    case 7: return go<7>(L, s);
    case 8: return go<8>(L, s);
    case 9: return go<9>(L, s);
    case 10: return go<10>(L, s);
    case 11: return go<11>(L, s);
    case 12: return go<12>(L, s);
    case 13: return go<13>(L, s);
    case 14: return go<14>(L, s);
    case 15: return go<15>(L, s);
    case 16: return go<16>(L, s);
    default: return hipErrorInvalidValue;
    }
}

namespace {

struct VegasWorkspace {
    double* grid = nullptr;          // [D][K+1]
    double* hist_partials = nullptr; // [blocks][D][K]
    double* hist = nullptr;          // [D][K]
    double* stats = nullptr;         // HYDRA_PHSP_STATS
    uint64_t partial_cap = 0;        // doubles
    double* host = nullptr;          // pinned: stats then hist
};

std::mutex g_vegas_mu;
std::map<std::pair<int, hipStream_t>, VegasWorkspace> g_vegas_ws;

void free_vegas(VegasWorkspace& w) {
    if (w.grid) (void)hipFree(w.grid);
    if (w.hist_partials) (void)hipFree(w.hist_partials);
    if (w.hist) (void)hipFree(w.hist);
    if (w.stats) (void)hipFree(w.stats);
    if (w.host) (void)hipHostFree(w.host);
    w = VegasWorkspace{};
}

int vegas_workspace(hipStream_t s, uint64_t partial_doubles, VegasWorkspace** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    std::lock_guard<std::mutex> lock(g_vegas_mu);
    VegasWorkspace& w = g_vegas_ws[std::make_pair(dev, s)];
    if (w.grid == nullptr) {
        const size_t tab = sizeof(double) * kVegasDMax * (kVegasKMax + 1);
        bool ok = hipMalloc(&w.grid, tab) == hipSuccess && hipMalloc(&w.hist, tab) == hipSuccess &&
                  hipMalloc(&w.stats, sizeof(double) * HYDRA_PHSP_STATS) == hipSuccess &&
                  hipHostMalloc(&w.host, sizeof(double) * HYDRA_PHSP_STATS + tab, hipHostMallocDefault) ==
                      hipSuccess;
        if (!ok) {
            free_vegas(w);
            return fail(HYDRA_PHSP_ENOMEM, "VEGAS workspace allocation failed");
        }
    }
    if (partial_doubles > w.partial_cap) {
        uint64_t cap = w.partial_cap ? w.partial_cap : (1u << 20);
        while (cap < partial_doubles) cap *= 2;
        if (w.hist_partials) (void)hipFree(w.hist_partials); // waits for the device
        w.hist_partials = nullptr;
        w.partial_cap = 0;
        if (hipMalloc(&w.hist_partials, sizeof(double) * cap) != hipSuccess)
            return fail(HYDRA_PHSP_ENOMEM, "VEGAS histogram workspace allocation failed");
        w.partial_cap = cap;
    }
    *out = &w;
    return HYDRA_PHSP_OK;
}

int check_box(const hydra_phsp_gauss_box* f, int bins) {
    if (f == nullptr) return fail(HYDRA_PHSP_EINVAL, "integrand is NULL");
    if (f->dim < 1 || f->dim > HYDRA_PHSP_VEGAS_DMAX) return fail(HYDRA_PHSP_EINVAL, "dim must be in [1, 16]");
    if (bins < 2 || bins > HYDRA_PHSP_VEGAS_KMAX) return fail(HYDRA_PHSP_EINVAL, "bins must be in [2, 128]");
    for (int d = 0; d < f->dim; ++d) {
        if (!std::isfinite(f->lo[d]) || !std::isfinite(f->hi[d]) || !(f->hi[d] > f->lo[d]))
            return fail(HYDRA_PHSP_EINVAL, "each box edge must be finite with hi > lo");
        if (!std::isfinite(f->mean[d]) || !std::isfinite(f->sigma[d]) || !(f->sigma[d] > 0.0))
            return fail(HYDRA_PHSP_EINVAL, "each Gaussian needs a finite mean and a finite sigma > 0");
    }
    return HYDRA_PHSP_OK;
}

// The integrand of an iteration: the box, and either the built-in Gaussian
// product (gauss) or a kernel compiled at run time from a user's function
// (user, with its parameters).
struct VegasIntegrand {
    int dim = 0;
    double lo[kVegasDMax] = {}, hi[kVegasDMax] = {};
    const hydra_phsp_gauss_box* gauss = nullptr;
    RtcKernel* user = nullptr;
    double upar[HYDRA_PHSP_USER_PARAMS] = {};
};

VegasIntegrand gauss_integrand(const hydra_phsp_gauss_box* f) {
    VegasIntegrand g;
    g.dim = f->dim;
    for (int d = 0; d < f->dim; ++d) {
        g.lo[d] = f->lo[d];
        g.hi[d] = f->hi[d];
    }
    g.gauss = f;
    return g;
}

// Refinement of one dimension's edges from its value^2 histogram h (see the
// header): smoothing, damped importance, equal-importance re-cut.
void refine_dim(int K, double* g, const double* h, double alpha) {
    std::vector<double> s((size_t)K), imp((size_t)K), cut((size_t)K + 1);
    double total = 0.0;
    for (int k = 0; k < K; ++k) {
        if (k == 0)
            s[0] = (h[0] + h[1]) / 2.0;
        else if (k == K - 1)
            s[k] = (h[K - 2] + h[K - 1]) / 2.0;
        else
            s[k] = (h[k - 1] + h[k] + h[k + 1]) / 3.0;
        total += s[k];
    }
    double imp_total = 0.0;
    for (int k = 0; k < K; ++k) {
        double r = 0.0;
        if (s[k] > 0.0) {
            const double ratio = total / s[k];
            r = ratio > 1.0 ? std::pow((1.0 - 1.0 / ratio) / std::log(ratio), alpha) : 1.0;
        }
        imp[k] = r;
        imp_total += r;
    }
    if (!(imp_total > 0.0)) return;
    const double quota = imp_total / (double)K;
    cut[0] = 0.0;
    int src = 0;              // old bin the next edge falls in
    double avail = imp[0];    // importance of that bin not yet assigned
    for (int e = 1; e < K; ++e) {
        double want = quota;
        while (want > avail && src < K - 1) {
            want -= avail;
            avail = imp[++src];
        }
        avail -= want;
        double f = imp[src] > 0.0 ? (imp[src] - avail) / imp[src] : 1.0;
        f = f < 0.0 ? 0.0 : (f > 1.0 ? 1.0 : f);
        cut[e] = g[src] + f * (g[src + 1] - g[src]);
    }
    cut[K] = 1.0;
    for (int e = 0; e <= K; ++e) g[e] = cut[e];
}

int vegas_iteration(const VegasIntegrand& f, int bins, const double* grid_dev, uint64_t calls, uint64_t seed,
                    uint32_t iteration, double* stats_dev, double* hist_dev, double* values_dev, hipStream_t s) {
    const int D = f.dim;
    hipFunction_t user_fn = nullptr;
    if (f.user != nullptr) {
        const int ust = rtc_function(f.user, 0, &user_fn);
        if (ust != HYDRA_PHSP_OK) return ust;
    }
    const uint64_t span = (uint64_t)kVegasBlock * (uint64_t)kVegasEpt;
    const uint64_t blocks = ceil_div(calls, span);
    if (blocks > 0xFFFFFFFFull / (uint64_t)kVegasBlock)
        return fail(HYDRA_PHSP_EINVAL, "calls too large for one launch (more than 2^32 - 1 threads)");
    const uint64_t groups = (blocks + kHistGroup - 1) / kHistGroup;
    if (groups > 65535) return fail(HYDRA_PHSP_EINVAL, "calls too large for the histogram reduction");
    VegasWorkspace* ws = nullptr;
    int st = vegas_workspace(s, hist_dev ? (blocks + groups) * (uint64_t)(D * bins) : 0, &ws);
    if (st != HYDRA_PHSP_OK) return st;
    Moments* partials = nullptr;
    st = block_partials(s, blocks, &partials);
    if (st != HYDRA_PHSP_OK) return st;
    VegasLaunch L;
    std::memset(&L, 0, sizeof(L));
    L.v.bins = bins;
    L.v.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
    L.v.k1 = (uint32_t)(seed >> 32);
    L.v.iteration = iteration;
    L.v.calls = calls;
    for (int d = 0; d < D; ++d) {
        L.v.lo[d] = f.lo[d];
        L.v.width[d] = f.hi[d] - f.lo[d];
        if (f.gauss != nullptr) {
            L.v.mu[d] = f.gauss->mean[d];
            L.v.inv_sigma[d] = 1.0 / f.gauss->sigma[d];
            L.v.norm[d] = 1.0 / (f.gauss->sigma[d] * 2.5066282746310002); // sqrt(2 pi)
        }
    }
    for (int k = 0; k < HYDRA_PHSP_USER_PARAMS; ++k) L.v.upar[k] = f.upar[k];
    L.v.grid = grid_dev;
    L.v.partials = partials;
    L.v.hist_partials = hist_dev ? ws->hist_partials : nullptr;
    L.v.values = values_dev;
    L.blocks = blocks;
    L.lds_bytes = sizeof(double) * ((size_t)D * (bins + 1) + (hist_dev ? (size_t)kVegasWaves * D * bins : 0));
    if (blocks > 0) {
        const long slot = timing_begin(s);
        hipError_t e = hipSuccess;
        if (user_fn != nullptr) {
            void* args[] = {&L.v};
            e = hipModuleLaunchKernel(user_fn, (unsigned)L.blocks, 1, 1, kVegasBlock, 1, 1, (unsigned)L.lds_bytes, s,
                                      args, nullptr);
        } else {
            e = launch_vegas(D, L, s);
        }
        timing_end(s, slot);
        if (e != hipSuccess) return fail_hip(e, "VEGAS kernel launch");
        if (hist_dev) {
            const int entries = D * bins;
            double* mid = ws->hist_partials + blocks * (uint64_t)entries;
            const unsigned ex = (unsigned)((entries + 255) / 256);
            hipLaunchKernelGGL(k_vegas_hist_groups, dim3(ex, (unsigned)groups), dim3(256), 0, s,
                               (const double*)ws->hist_partials, blocks, entries, mid);
            e = hipGetLastError();
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_vegas_hist_sum, dim3(ex), dim3(256), 0, s, (const double*)mid, groups, entries,
                                   hist_dev);
                e = hipGetLastError();
            }
            if (e != hipSuccess) return fail_hip(e, "VEGAS histogram kernel launch");
        }
    }
    return merge_partials(s, partials, blocks, stats_dev);
}

} // namespace

int release_vegas_workspaces() {
    std::lock_guard<std::mutex> lock(g_vegas_mu);
    for (auto& kv : g_vegas_ws) free_vegas(kv.second);
    g_vegas_ws.clear();
    return HYDRA_PHSP_OK;
}

} // namespace hphsp

using namespace hphsp;

struct hydra_phsp_user_integrand {
    int dim = 0;
    RtcKernel* kernel = nullptr;
};

namespace hphsp {
namespace {

int check_user(const hydra_phsp_user_integrand* f, const double* lo, const double* hi, const double* params,
               int n_params, int bins) {
    if (f == nullptr) return fail(HYDRA_PHSP_EINVAL, "integrand is NULL");
    if (bins < 2 || bins > HYDRA_PHSP_VEGAS_KMAX) return fail(HYDRA_PHSP_EINVAL, "bins must be in [2, 128]");
    if (lo == nullptr || hi == nullptr) return fail(HYDRA_PHSP_EINVAL, "lo_host and hi_host are required");
    for (int d = 0; d < f->dim; ++d)
        if (!std::isfinite(lo[d]) || !std::isfinite(hi[d]) || !(hi[d] > lo[d]))
            return fail(HYDRA_PHSP_EINVAL, "each box edge must be finite with hi > lo");
    if (n_params < 0 || n_params > HYDRA_PHSP_USER_PARAMS)
        return fail(HYDRA_PHSP_EINVAL, "n_params must be in [0, HYDRA_PHSP_USER_PARAMS]");
    if (n_params > 0 && params == nullptr) return fail(HYDRA_PHSP_EINVAL, "params_host is NULL");
    return HYDRA_PHSP_OK;
}

VegasIntegrand user_integrand(const hydra_phsp_user_integrand* f, const double* lo, const double* hi,
                              const double* params, int n_params) {
    VegasIntegrand g;
    g.dim = f->dim;
    for (int d = 0; d < f->dim; ++d) {
        g.lo[d] = lo[d];
        g.hi[d] = hi[d];
    }
    g.user = f->kernel;
    for (int k = 0; k < n_params; ++k) g.upar[k] = params[k];
    return g;
}

int check_iteration_buffers(const double* grid_dev, uint64_t calls, const double* stats_dev, const double* hist_dev,
                            const double* values_dev) {
    if (grid_dev == nullptr || stats_dev == nullptr) return fail(HYDRA_PHSP_EINVAL, "grid_dev and stats_dev are required");
    if (calls < 2) return fail(HYDRA_PHSP_EINVAL, "need calls >= 2 (the error estimate needs two samples)");
    if ((uintptr_t)grid_dev % 8 || (uintptr_t)stats_dev % 8 || (uintptr_t)hist_dev % 8 || (uintptr_t)values_dev % 8)
        return fail(HYDRA_PHSP_EINVAL, "device pointers must be 8-byte aligned");
    return HYDRA_PHSP_OK;
}

// The whole integration (see hydra_phsp_vegas), for either kind of integrand.
int vegas_run(const VegasIntegrand& f, int bins, uint64_t calls, int warmup, int iterations, double alpha,
              uint64_t seed, double* grid_host, double* result, double* error, double* chi2_dof, hipStream_t s) {
    if (calls < 2 || warmup < 0 || iterations < 1) return fail(HYDRA_PHSP_EINVAL, "need calls >= 2 and iterations >= 1");
    if (result == nullptr || error == nullptr || chi2_dof == nullptr)
        return fail(HYDRA_PHSP_EINVAL, "result, error and chi2_dof are required");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(HYDRA_PHSP_EINVAL, "alpha must be finite and >= 0");
    const int D = f.dim, K = bins;
    std::vector<double> grid((size_t)D * (K + 1));
    for (int d = 0; d < D; ++d)
        for (int k = 0; k <= K; ++k) grid[(size_t)d * (K + 1) + k] = grid_host ? grid_host[(size_t)d * (K + 1) + k] : (double)k / K;
    VegasWorkspace* ws = nullptr;
    int st = vegas_workspace(s, 0, &ws);
    if (st != HYDRA_PHSP_OK) return st;
    std::vector<std::pair<double, double>> est; // (mean, 1/sigma^2) of the estimating iterations
    for (int t = 0; t < warmup + iterations; ++t) {
        hipError_t e = hipMemcpyAsync(ws->grid, grid.data(), sizeof(double) * grid.size(), hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return fail_hip(e, "VEGAS grid upload");
        st = vegas_iteration(f, K, ws->grid, calls, seed, (uint32_t)t, ws->stats, ws->hist, nullptr, s);
        if (st != HYDRA_PHSP_OK) return st;
        e = hipMemcpyAsync(ws->host, ws->stats, sizeof(double) * HYDRA_PHSP_STATS, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(ws->host + HYDRA_PHSP_STATS, ws->hist, sizeof(double) * D * K, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return fail_hip(e, "VEGAS iteration readback");
        const double mean = ws->host[1], sig = ws->host[3];
        if (t >= warmup && sig > 0.0) est.emplace_back(mean, 1.0 / (sig * sig));
        for (int d = 0; d < D; ++d)
            refine_dim(K, grid.data() + (size_t)d * (K + 1), ws->host + HYDRA_PHSP_STATS + (size_t)d * K, alpha);
    }
    double sw = 0.0, swx = 0.0;
    for (const auto& m : est) {
        sw += m.second;
        swx += m.second * m.first;
    }
    if (!(sw > 0.0)) return fail(HYDRA_PHSP_EINVAL, "no iteration had a non-zero variance");
    const double res = swx / sw;
    double chi = 0.0;
    for (const auto& m : est) chi += m.second * (m.first - res) * (m.first - res);
    *result = res;
    *error = 1.0 / std::sqrt(sw);
    *chi2_dof = est.size() > 1 ? chi / (double)(est.size() - 1) : 0.0;
    if (grid_host)
        for (size_t i = 0; i < grid.size(); ++i) grid_host[i] = grid[i];
    return HYDRA_PHSP_OK;
}

std::string integrand_source(const char* user, int dim) {
    std::string s;
    s += "#define HYDRA_PHSP_DIM " + std::to_string(dim) + "\n";
    s += "#include \"phsp_vegas.hpp\"\n";
    // the user's function is inlined into the sample loop (x is the sample's
    // coordinates in registers)
    s += "__device__ __attribute__((always_inline)) double hydra_phsp_user_integrand(const double* x, "
         "const double* par);\n";
    s += "#line 1 \"user_integrand\"\n";
    s += user;
    s += "\n#line 1 \"user_integrand_kernel\"\n";
    // the integrand type of the VEGAS kernel: coordinates and Jacobian per
    // dimension, then the user's function times the Jacobian
    s += "struct hydra_phsp_user_integrand_f {\n"
         "    double x[HYDRA_PHSP_DIM];\n"
         "    double jac = 1.0;\n"
         "    __device__ __forceinline__ void dim(const hphsp::VegasArgs&, int d, double xd, double j) {\n"
         "        x[d] = xd;\n"
         "        jac = jac * j;\n"
         "    }\n"
         "    __device__ __forceinline__ double value(const hphsp::VegasArgs& v) const {\n"
         "        return hydra_phsp_user_integrand(x, v.upar) * jac;\n"
         "    }\n"
         "};\n";
    return s;
}

} // namespace
} // namespace hphsp

extern "C" {

int hydra_phsp_vegas_iteration(const hydra_phsp_gauss_box* f, int bins, const double* grid_dev, uint64_t calls,
                               uint64_t seed, uint32_t iteration, double* stats_dev, double* hist_dev,
                               double* values_dev, void* stream) {
    MarkerRange marker("hydra_phsp_vegas_iteration");
    int st = check_box(f, bins);
    if (st != HYDRA_PHSP_OK) return st;
    st = check_iteration_buffers(grid_dev, calls, stats_dev, hist_dev, values_dev);
    if (st != HYDRA_PHSP_OK) return st;
    return vegas_iteration(gauss_integrand(f), bins, grid_dev, calls, seed, iteration, stats_dev, hist_dev, values_dev,
                           (hipStream_t)stream);
}

int hydra_phsp_vegas_refine(int dim, int bins, double* grid_host, const double* hist_host, double alpha) {
    if (dim < 1 || dim > HYDRA_PHSP_VEGAS_DMAX || bins < 2 || bins > HYDRA_PHSP_VEGAS_KMAX)
        return fail(HYDRA_PHSP_EINVAL, "dim must be in [1, 16] and bins in [2, 128]");
    if (grid_host == nullptr || hist_host == nullptr) return fail(HYDRA_PHSP_EINVAL, "grid and histogram are required");
    if (!(alpha >= 0.0) || !std::isfinite(alpha)) return fail(HYDRA_PHSP_EINVAL, "alpha must be finite and >= 0");
    for (int d = 0; d < dim; ++d) refine_dim(bins, grid_host + (size_t)d * (bins + 1), hist_host + (size_t)d * bins, alpha);
    return HYDRA_PHSP_OK;
}

int hydra_phsp_vegas(const hydra_phsp_gauss_box* f, int bins, uint64_t calls, int warmup, int iterations,
                     double alpha, uint64_t seed, double* grid_host, double* result, double* error,
                     double* chi2_dof, void* stream) {
    MarkerRange marker("hydra_phsp_vegas");
    const int st = check_box(f, bins);
    if (st != HYDRA_PHSP_OK) return st;
    return vegas_run(gauss_integrand(f), bins, calls, warmup, iterations, alpha, seed, grid_host, result, error,
                     chi2_dof, (hipStream_t)stream);
}

int hydra_phsp_user_integrand_create(const char* source_host, int dim, hydra_phsp_user_integrand** integrand_out) {
    if (integrand_out == nullptr) return fail(HYDRA_PHSP_EINVAL, "integrand_out is NULL");
    *integrand_out = nullptr;
    if (source_host == nullptr) return fail(HYDRA_PHSP_EINVAL, "source_host is NULL");
    if (dim < 1 || dim > HYDRA_PHSP_VEGAS_DMAX) return fail(HYDRA_PHSP_EINVAL, "dim must be in [1, 16]");
    const std::string kernel = "hphsp::k_vegas<" + std::to_string(dim) + ", hydra_phsp_user_integrand_f>";
    RtcKernel* k = nullptr;
    const int st = rtc_compile(integrand_source(source_host, dim), {RtcName{kernel, true}}, "user integrand", &k);
    if (st != HYDRA_PHSP_OK) return st;
    auto* f = new hydra_phsp_user_integrand();
    f->dim = dim;
    f->kernel = k;
    *integrand_out = f;
    return HYDRA_PHSP_OK;
}

int hydra_phsp_user_integrand_destroy(hydra_phsp_user_integrand* integrand) {
    if (integrand == nullptr) return fail(HYDRA_PHSP_EINVAL, "integrand is NULL");
    const int st = rtc_destroy(integrand->kernel);
    delete integrand;
    return st;
}

int hydra_phsp_vegas_user_iteration(hydra_phsp_user_integrand* f, const double* lo_host, const double* hi_host,
                                    const double* params_host, int n_params, int bins, const double* grid_dev,
                                    uint64_t calls, uint64_t seed, uint32_t iteration, double* stats_dev,
                                    double* hist_dev, double* values_dev, void* stream) {
    MarkerRange marker("hydra_phsp_vegas_user_iteration");
    int st = check_user(f, lo_host, hi_host, params_host, n_params, bins);
    if (st != HYDRA_PHSP_OK) return st;
    st = check_iteration_buffers(grid_dev, calls, stats_dev, hist_dev, values_dev);
    if (st != HYDRA_PHSP_OK) return st;
    return vegas_iteration(user_integrand(f, lo_host, hi_host, params_host, n_params), bins, grid_dev, calls, seed,
                           iteration, stats_dev, hist_dev, values_dev, (hipStream_t)stream);
}

int hydra_phsp_vegas_user(hydra_phsp_user_integrand* f, const double* lo_host, const double* hi_host,
                          const double* params_host, int n_params, int bins, uint64_t calls, int warmup,
                          int iterations, double alpha, uint64_t seed, double* grid_host, double* result,
                          double* error, double* chi2_dof, void* stream) {
    MarkerRange marker("hydra_phsp_vegas_user");
    const int st = check_user(f, lo_host, hi_host, params_host, n_params, bins);
    if (st != HYDRA_PHSP_OK) return st;
    return vegas_run(user_integrand(f, lo_host, hi_host, params_host, n_params), bins, calls, warmup, iterations,
                     alpha, seed, grid_host, result, error, chi2_dof, (hipStream_t)stream);
}

} // extern "C"

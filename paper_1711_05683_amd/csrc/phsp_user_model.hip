// phsp_user_model.hip -- kernels compiled at run time from user code, and model
// evaluation with a user's intensity function.
//
// Hydra evaluates user code passed as functors with parameters (sec. 3.1 of
// arXiv:1711.05683) and lists model evaluation over phase space among the
// generator's uses (sec. 4.2).  Here the user hands over HIP device source; the
// library compiles it with hiprtc for gfx950, with its own compiler flags,
// together with the generator's kernel headers (embedded in the library at
// build time), into one kernel in which the user's function is inlined where
// the built-in one would be.  The code object is compiled once and loaded on
// each device at its first use there.  For model evaluation the source defines
//   double hydra_phsp_user_intensity(const double* e, const double* px,
//                                    const double* py, const double* pz,
//                                    const double* par)
// over the N daughters' four-momenta; the VEGAS integrands of
// phsp_vegas_api.hip use the same machinery.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "hydra_phsp.h"
#include "hydra_phsp_model.h"
#include "phsp_api_internal.hpp"
#include "phsp_model.hpp"

namespace hphsp {

namespace {

#include "phsp_rtc_sources.inc"

// The kernel headers include <hip/hip_runtime.h>; under hiprtc the device side
// of HIP is built in, and only the two host types named by the headers'
// launcher declarations are missing.
const char* const kRtcRuntimeStub =
    "#pragma once\n"
    "typedef int hipError_t;\n"
    "typedef struct ihipStream_t* hipStream_t;\n";

constexpr int kMaxDevices = 64;
constexpr size_t kMaxLogBytes = 8192;

} // namespace

constexpr int kMaxRtcKernels = 4;

struct RtcKernel {
    std::vector<char> code;            // gfx950 code object
    std::vector<std::string> symbols;  // the kernels' (lowered) names in it
    std::mutex mu;
    hipModule_t module[kMaxDevices] = {};
    hipFunction_t fn[kMaxDevices][kMaxRtcKernels] = {};
};

int rtc_compile(const std::string& source, const std::vector<RtcName>& kernels, const char* what, RtcKernel** out) {
    *out = nullptr;
    std::vector<const char*> names, texts;
    names.push_back("hip/hip_runtime.h");
    texts.push_back(kRtcRuntimeStub);
    for (int i = 0; i < kRtcHeaders; ++i) {
        names.push_back(kRtcHeaderNames[i]);
        texts.push_back(kRtcHeaderSources[i]);
    }
    hiprtcProgram prog = nullptr;
    hiprtcResult r = hiprtcCreateProgram(&prog, source.c_str(), "user.hip", (int)names.size(), texts.data(),
                                         names.data());
    if (r != HIPRTC_SUCCESS)
        return fail(HYDRA_PHSP_EDEVICE, std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r));
    if (kernels.empty() || kernels.size() > (size_t)kMaxRtcKernels) {
        (void)hiprtcDestroyProgram(&prog);
        return fail(HYDRA_PHSP_EINVAL, "run-time module kernel count out of range");
    }
    for (const RtcName& k : kernels) {
        if (!k.expression) continue;
        r = hiprtcAddNameExpression(prog, k.name.c_str());
        if (r != HIPRTC_SUCCESS) {
            (void)hiprtcDestroyProgram(&prog);
            return fail(HYDRA_PHSP_EDEVICE, std::string("hiprtcAddNameExpression: ") + hiprtcGetErrorString(r));
        }
    }
    // the library's own flags: gfx950, no contraction (explicit fma only), no
    // packed FP32
    const char* opts[] = {"--offload-arch=gfx950", "-O3",     "-std=c++17",      "-ffp-contract=off",
                          "-Xclang",               "-target-feature", "-Xclang", "-packed-fp32-ops"};
    r = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
    if (r != HIPRTC_SUCCESS) {
        size_t n = 0;
        std::string log;
        if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 0) {
            log.resize(n);
            if (hiprtcGetProgramLog(prog, &log[0]) != HIPRTC_SUCCESS) log.clear();
            if (log.size() > kMaxLogBytes) log.resize(kMaxLogBytes);
        }
        (void)hiprtcDestroyProgram(&prog);
        if (r == HIPRTC_ERROR_COMPILATION || r == HIPRTC_ERROR_LINKING)
            return fail(HYDRA_PHSP_EINVAL, std::string(what) + " does not compile: " + log);
        return fail(HYDRA_PHSP_EDEVICE, std::string("hiprtcCompileProgram: ") + hiprtcGetErrorString(r));
    }
    auto* k = new RtcKernel();
    for (const RtcName& kn : kernels) {
        if (!kn.expression) {
            k->symbols.push_back(kn.name);
            continue;
        }
        const char* lowered = nullptr;
        r = hiprtcGetLoweredName(prog, kn.name.c_str(), &lowered);
        if (r != HIPRTC_SUCCESS || lowered == nullptr) {
            (void)hiprtcDestroyProgram(&prog);
            delete k;
            return fail(HYDRA_PHSP_EDEVICE, "hiprtcGetLoweredName failed");
        }
        k->symbols.push_back(lowered);
    }
    size_t size = 0;
    r = hiprtcGetCodeSize(prog, &size);
    if (r == HIPRTC_SUCCESS && size > 0) {
        k->code.resize(size);
        r = hiprtcGetCode(prog, k->code.data());
    }
    (void)hiprtcDestroyProgram(&prog);
    if (r != HIPRTC_SUCCESS || size == 0) {
        delete k;
        return fail(HYDRA_PHSP_EDEVICE, "hiprtc produced no code object");
    }
    *out = k;
    return HYDRA_PHSP_OK;
}

int rtc_function(RtcKernel* k, int which, hipFunction_t* out) {
    if (which < 0 || which >= (int)k->symbols.size()) return fail(HYDRA_PHSP_EINVAL, "run-time kernel index");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(HYDRA_PHSP_EINVAL, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(k->mu);
    if (k->module[dev] == nullptr) {
        hipModule_t mod = nullptr;
        e = hipModuleLoadData(&mod, k->code.data());
        if (e != hipSuccess) return fail_hip(e, "hipModuleLoadData(run-time kernel)");
        hipFunction_t fns[kMaxRtcKernels] = {};
        for (size_t i = 0; i < k->symbols.size() && e == hipSuccess; ++i)
            e = hipModuleGetFunction(&fns[i], mod, k->symbols[i].c_str());
        if (e != hipSuccess) {
            (void)hipModuleUnload(mod);
            return fail_hip(e, "hipModuleGetFunction(run-time kernel)");
        }
        k->module[dev] = mod;
        for (int i = 0; i < kMaxRtcKernels; ++i) k->fn[dev][i] = fns[i];
    }
    *out = k->fn[dev][which];
    return HYDRA_PHSP_OK;
}

int rtc_destroy(RtcKernel* k) {
    int st = HYDRA_PHSP_OK;
    int cur = 0;
    const bool have_cur = hipGetDevice(&cur) == hipSuccess;
    for (int d = 0; d < kMaxDevices; ++d) {
        if (k->module[d] == nullptr) continue;
        // the module's kernels may still be queued: wait for the device first
        if (hipSetDevice(d) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
            hipModuleUnload(k->module[d]) != hipSuccess)
            st = fail(HYDRA_PHSP_EDEVICE, "run-time kernel unload failed");
    }
    if (have_cur) (void)hipSetDevice(cur);
    delete k;
    return st;
}

namespace {

// Kernel arguments after the model's: the user's parameters, by value.
struct UserParams {
    double p[HYDRA_PHSP_USER_PARAMS];
};

std::string model_source(const char* user, int n) {
    std::string s;
    s += "#define HYDRA_PHSP_N " + std::to_string(n) + "\n";
    s += "#include \"phsp_model.hpp\"\n";
    s += "#include \"phsp_unweight.hpp\"\n";
    // the user's function is inlined into the event loop (its array arguments
    // are the event's registers)
    s += "__device__ __attribute__((always_inline)) double hydra_phsp_user_intensity(const double* e, "
         "const double* px, const double* py, const double* pz, const double* par);\n";
    s += "#line 1 \"user_intensity\"\n";
    s += user;
    s += "\n#line 1 \"user_model_kernel\"\n";
    s += "struct hydra_phsp_user_params { double p[" + std::to_string(HYDRA_PHSP_USER_PARAMS) + "]; };\n";
    s += "extern \"C\" __global__ __launch_bounds__(256) void hydra_phsp_user_model_kernel("
         "const hphsp::ModelArgs m, const hydra_phsp_user_params par) {\n"
         "    hphsp::model_block<HYDRA_PHSP_N>(m, [&](const hphsp::Event<HYDRA_PHSP_N, double>& ev) {\n"
         "        return hydra_phsp_user_intensity(ev.e, ev.x, ev.y, ev.z, par.p);\n"
         "    });\n"
         "}\n";
    // the intensity type of the unweighted count and maximum passes
    s += "struct hydra_phsp_user_intensity_u {\n"
         "    static constexpr bool kKinematics = true;\n"
         "    template <int N>\n"
         "    __device__ __forceinline__ double operator()(const hphsp::UnwArgs& u,\n"
         "                                                 const hphsp::Event<N, double>& ev) const {\n"
         "        return hydra_phsp_user_intensity(ev.e, ev.x, ev.y, ev.z, u.upar);\n"
         "    }\n"
         "};\n";
    return s;
}

// The kernels of a user model's module: model evaluation, then the unweighted
// maximum and count passes.
std::vector<RtcName> model_kernels(int n) {
    const std::string t = "<" + std::to_string(n) + ", hydra_phsp_user_intensity_u>";
    return {RtcName{"hydra_phsp_user_model_kernel", false}, RtcName{"hphsp::k_unw_max" + t, true},
            RtcName{"hphsp::k_unw_count" + t, true}};
}

} // namespace
} // namespace hphsp

using namespace hphsp;

struct hydra_phsp_user_model {
    int n = 0;
    RtcKernel* kernel = nullptr;
};

namespace hphsp {

RtcKernel* user_model_kernels(const hydra_phsp_user_model* model, int* n_daughters) {
    *n_daughters = model->n;
    return model->kernel;
}

} // namespace hphsp

extern "C" int hydra_phsp_user_model_create(const char* source_host, int n_daughters,
                                            hydra_phsp_user_model** model_out) {
    if (model_out == nullptr) return fail(HYDRA_PHSP_EINVAL, "model_out is NULL");
    *model_out = nullptr;
    if (source_host == nullptr) return fail(HYDRA_PHSP_EINVAL, "source_host is NULL");
    if (n_daughters < 2 || n_daughters > kNMax) return fail(HYDRA_PHSP_EINVAL, "n_daughters must be in [2, 10]");
    RtcKernel* k = nullptr;
    const int st = rtc_compile(model_source(source_host, n_daughters), model_kernels(n_daughters), "user model", &k);
    if (st != HYDRA_PHSP_OK) return st;
    auto* um = new hydra_phsp_user_model();
    um->n = n_daughters;
    um->kernel = k;
    *model_out = um;
    return HYDRA_PHSP_OK;
}

extern "C" int hydra_phsp_user_model_destroy(hydra_phsp_user_model* model) {
    if (model == nullptr) return fail(HYDRA_PHSP_EINVAL, "model is NULL");
    const int st = rtc_destroy(model->kernel);
    delete model;
    return st;
}

extern "C" int hydra_phsp_user_model_daughters(const hydra_phsp_user_model* model) {
    return model == nullptr ? fail(HYDRA_PHSP_EINVAL, "model is NULL") : model->n;
}

extern "C" int hydra_phsp_integrate_user_model(hydra_phsp_user_model* model, double parent_mass,
                                               const double* masses_host, const double* params_host,
                                               int n_params, uint64_t nevents, uint64_t seed, uint32_t stream_id,
                                               uint64_t event_offset, double* values_dev, double* stats_dev,
                                               void* stream) {
    MarkerRange marker("hydra_phsp_integrate_user_model");
    if (model == nullptr) return fail(HYDRA_PHSP_EINVAL, "model is NULL");
    Channel ch;
    int st = make_channel(parent_mass, masses_host, model->n, &ch);
    if (st != HYDRA_PHSP_OK) return st;
    if (n_params < 0 || n_params > HYDRA_PHSP_USER_PARAMS)
        return fail(HYDRA_PHSP_EINVAL, "n_params must be in [0, HYDRA_PHSP_USER_PARAMS]");
    if (n_params > 0 && params_host == nullptr) return fail(HYDRA_PHSP_EINVAL, "params_host is NULL");
    if (stats_dev == nullptr) return fail(HYDRA_PHSP_EINVAL, "stats_dev is required");
    if ((uintptr_t)values_dev % sizeof(double) != 0 || (uintptr_t)stats_dev % sizeof(double) != 0)
        return fail(HYDRA_PHSP_EINVAL, "device pointers must be aligned to their element size");
    UserParams par;
    std::memset(&par, 0, sizeof(par));
    for (int k = 0; k < n_params; ++k) par.p[k] = params_host[k];
    const uint64_t span = (uint64_t)kBlock * (uint64_t)kModelEpt;
    const uint64_t blocks = ceil_div(nevents, span);
    if (blocks > 0xFFFFFFFFull / (uint64_t)kBlock)
        return fail(HYDRA_PHSP_EINVAL, "nevents too large for one launch (more than 2^32 - 1 threads)");
    hipFunction_t fn = nullptr;
    st = rtc_function(model->kernel, kUserModelKernel, &fn);
    if (st != HYDRA_PHSP_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Moments* partials = nullptr;
    st = block_partials(s, blocks, &partials);
    if (st != HYDRA_PHSP_OK) return st;
    const double2* trig = nullptr;
    st = trig_table(&trig);
    if (st != HYDRA_PHSP_OK) return st;
    ModelArgs m;
    std::memset(&m, 0, sizeof(m));
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
        void* args[] = {&m, &par};
        const long slot = timing_begin(s);
        const hipError_t e =
            hipModuleLaunchKernel(fn, (unsigned)blocks, 1, 1, kBlock, 1, 1, 0, s, args, nullptr);
        timing_end(s, slot);
        if (e != hipSuccess) return fail_hip(e, "user model kernel launch");
    }
    return merge_partials(s, partials, blocks, stats_dev);
}

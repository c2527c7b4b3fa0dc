// phsp_api_internal.hpp -- host helpers shared by the library's C-ABI units.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <string>
#include <vector>

#include "phsp_device.hpp"
#include "phsp_reduce.hpp"

struct hydra_phsp_breit_wigner;
struct hydra_phsp_user_model;

namespace hphsp {

// Named host range around one ABI call that enqueues device work, visible to
// rocprofv3 --marker-trace beside the kernels it launched; a push and a pop,
// cheap when no tool listens.  (The allocation-free entry point has none.)
class MarkerRange {
  public:
    explicit MarkerRange(const char* name) { roctxRangePushA(name); }
    ~MarkerRange() { roctxRangePop(); }
    MarkerRange(const MarkerRange&) = delete;
    MarkerRange& operator=(const MarkerRange&) = delete;
};

// ceil(a / b) for b > 0, without the overflow of (a + b - 1) / b near 2^64
// (event counts come from callers unchecked).
inline uint64_t ceil_div(uint64_t a, uint64_t b) { return a / b + (a % b != 0 ? 1 : 0); }

int fail(int status, const std::string& msg);
int fail_hip(hipError_t e, const char* what);
// Validate (M, masses, n) and fill the per-channel constants.
int make_channel(double M, const double* masses, int n, Channel* out);
// Validate a parent four-vector of mass M and fill its boost.
int make_frame(double M, const double* p4, Frame* f);
// Single-channel launch with a given events-per-thread (0 = default).
int run_single(const Channel& ch, int n, int pmode, const Frame* frame, const double* parent_dev,
               uint64_t ld_parent, uint64_t nevents, uint64_t seed, uint32_t sid, uint64_t offset,
               int mode, void* out, uint64_t ld, double* weights, double* stats_dev, hipStream_t stream,
               int ept_override);
// Events per thread a single-channel launch uses for (mode, n, parent mode,
// staged layout), after the process-wide override.
int single_channel_ept(int mode, int n, int pmode, bool staged);
// The stream's block-partials buffer, grown to at least `blocks` entries (valid
// until the next call on the stream that grows it).
int block_partials(hipStream_t stream, uint64_t blocks, Moments** partials);
// Two-stage fixed-order merge of `blocks` partials into HYDRA_PHSP_STATS doubles.
int merge_partials(hipStream_t stream, const Moments* partials, uint64_t blocks, double* stats_dev);
int release_workspaces();
int release_unweight_workspaces();
int release_vegas_workspaces();
int release_batch_slots();
// The device's (cos, sin) table used by the FP64 kernels (created on first use).
int trig_table(const double2** out);
// Kernels compiled at run time (user intensities and integrands): hiprtc for
// gfx950 with the library's flags against its own kernel headers (embedded at
// build time), the code object kept and loaded on each device at its first use.
struct RtcKernel;
struct RtcName {
    std::string name; // the kernel's extern "C" name, or a C++ name expression
    bool expression;  // (then hiprtc reports its lowered name)
};
// Compile `source` with the kernels `names`.  A source that does not compile
// fails with EINVAL and "<what> does not compile: <log>".
int rtc_compile(const std::string& source, const std::vector<RtcName>& names, const char* what, RtcKernel** out);
// Kernel `which` (its index in `names`) on the current device (loading the code
// object there at the first call).
int rtc_function(RtcKernel* k, int which, hipFunction_t* fn);
// Waits for the devices it was loaded on, unloads and frees it.
int rtc_destroy(RtcKernel* k);
// The kernels of a user model's module, by index, and the model's module.
enum { kUserModelKernel = 0, kUserModelUnwMax = 1, kUserModelUnwCount = 2 };
RtcKernel* user_model_kernels(const hydra_phsp_user_model* model, int* n_daughters);
// Validate up to HYDRA_PHSP_MAX_BW Breit-Wigner factors of an N-body model and
// copy them into the kernels' form.
struct BwFactors;
int make_bw_factors(const hydra_phsp_breit_wigner* res, int n_res, int n_daughters, BwFactors* out);
// Benchmark timing brackets around a kernel launch (slot -1: timing off).
long timing_begin(hipStream_t stream);
void timing_end(hipStream_t stream, long slot);

} // namespace hphsp

/*
 * hydra_phsp.h -- C ABI of the MI355X (gfx950) phase-space Monte Carlo library.
 *
 * The library generates and integrates N-body phase space with the
 * Raubold-Lynch method (arXiv:1711.05683, sec. 4.2 "Phase-Space Monte Carlo"):
 * a parent of given four-momentum decays to n daughters without intermediate
 * resonances; every event carries the full kinematics of the daughters and a
 * weight, and the mean weight estimates the n-body phase-space volume.
 *
 * Conventions (the paper fixes the problem and the interface of listing
 * "lst:phsp"; the rest are the readings documented with the library):
 *   - four-vectors are (E, px, py, pz): the listing builds the parent at rest
 *     as Vector4R(mass, 0, 0, 0);
 *   - the parent mass and the daughter masses are fixed per call, as in the
 *     listing's PhaseSpace<N>(mass, masses) object; the parent four-vector is
 *     given at generation time, as in Generate(Mother, begin, end);
 *   - measure: prod_i d^3p_i/(2E_i) delta^4(P - sum_i p_i), no factors of 2*pi;
 *     the mean weight is the n-body volume in this measure;
 *   - random numbers: Philox4x32-10, key = seed, counter =
 *     (g mod 2^32, g div 2^32, call index, stream_id) for global event index
 *     g = event_offset + e.  Results depend only on (seed, stream_id, g), so
 *     chunked, sharded and resumed runs are bit-identical to a single run;
 *   - daughter 0 is the innermost: the masses of the subsystems {0..i} are
 *     drawn first, then the levels run top down: level i splits {0..i+1} into
 *     daughter i+1 and {0..i}, back to back in the rest frame of {0..i+1}, and
 *     boosts both into the parent's rest frame (one boost per daughter).
 *
 * Memory: pointers named *_dev are device pointers (e.g. from torch tensors),
 * owned by the caller and left untouched outside the call; *_host pointers are
 * host memory read during the call only.  Momenta are structure-of-arrays:
 * component mu (0=E, 1=px, 2=py, 3=pz) of daughter d for event e is at
 * p4_out_dev[(4*d + mu)*ld + e], with ld >= nevents.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).
 * Calls documented as asynchronous only enqueue work on it; a device fault
 * surfaces at the next synchronising call as HYDRA_PHSP_EDEVICE.  Calls on
 * different streams may run concurrently from different host threads.
 *
 * Errors: every entry point returns a status code; all argument checks happen
 * before any work is enqueued, so a failed call has no effect on the device.
 * hydra_phsp_strerror() names a code, hydra_phsp_last_error() gives the text
 * of the calling thread's most recent failure.
 */
#ifndef HYDRA_PHSP_H
#define HYDRA_PHSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HYDRA_PHSP_NMAX 10 /* largest number of daughters */
#define HYDRA_PHSP_ABI_VERSION 1

enum {
    HYDRA_PHSP_OK = 0,
    HYDRA_PHSP_EINVAL = -1,      /* bad argument: N outside [2, NMAX], null pointer, ld < nevents, ... */
    HYDRA_PHSP_EKINEMATICS = -2, /* parent mass not above the sum of daughter masses */
    HYDRA_PHSP_ENOMEM = -3,      /* device or host allocation failed / budget exceeded */
    HYDRA_PHSP_EDEVICE = -4,     /* a HIP runtime error (text in hydra_phsp_last_error) */
    HYDRA_PHSP_EAGAIN = -5,      /* serving: result not ready yet */
    HYDRA_PHSP_ENOTFOUND = -6    /* serving: unknown or already collected request id */
};

/* Integral statistics written to a device buffer of HYDRA_PHSP_STATS doubles:
 * [0] n (number of events), [1] mean weight (the volume estimate),
 * [2] M2 = sum over events of (w - mean)^2, [3] sigma = sqrt(M2 / ((n-1) n)),
 * the standard error of the mean (0 when n < 2). */
#define HYDRA_PHSP_STATS 4

/* Parameters a user function compiled at run time receives (par[0..15]): the
 * model intensities of hydra_phsp_model.h and the VEGAS integrands of
 * hydra_phsp_vegas.h. */
#define HYDRA_PHSP_USER_PARAMS 16

/* ------------------------------------------------------------------------ */
/* Plain FP64 path                                                           */
/* ------------------------------------------------------------------------ */

/* Generate `nevents` weighted phase-space events (sec. 4.2; listing lst:phsp's
 * Generate(Mother, begin, end)).  Asynchronous on `stream`.
 *
 *   parent_mass      M > 0, the decaying particle's mass.
 *   masses_host      n_daughters masses >= 0 (host), sum < M (else EKINEMATICS).
 *   n_daughters      2 .. HYDRA_PHSP_NMAX.
 *   parent_p4_host   NULL: parent at rest.  Else 4 doubles (E, px, py, pz) of one
 *                    parent applied to every event (boost eta = p/M, gamma = E/M).
 *   parent_p4_dev    NULL, or per-event parents (SoA, component mu of event e at
 *                    parent_p4_dev[mu*ld_parent + e], ld_parent >= nevents); the
 *                    decay uses M and each parent only for its boost, so every
 *                    parent's invariant mass must equal M.  At most one of
 *                    parent_p4_host / parent_p4_dev may be non-NULL.
 *                    Sequential decays (sec. 4.2): daughter d of an earlier
 *                    FP64 call is p4_out_dev + 4*d*ld of that call with
 *                    ld_parent = its ld, read in place, with M = its mass and
 *                    another stream_id (or seed) so the two stages draw
 *                    independent uniforms.
 *   nevents          number of events (0 is a no-op that still writes stats).
 *   seed, stream_id  Philox key and counter word 3.
 *   event_offset     global index of the first event.
 *   p4_out_dev       [n_daughters][4][ld] doubles (device).  Any ld >= nevents
 *                    works; a 128-byte aligned p4_out_dev with ld a multiple of
 *                    16 (32 for the FP32 outputs of the mixed path) starts every
 *                    column on a cache line, so every wave's stores are whole-line
 *                    writes.  Misaligned columns turn them into partial-line
 *                    writes, measured at up to ~40% less write bandwidth.
 *   weights_dev      [nevents] doubles (device).
 *   stats_dev        NULL, or HYDRA_PHSP_STATS doubles (device) receiving the
 *                    fused integral of this call's weights.
 */
int hydra_phsp_generate(double parent_mass, const double *masses_host, int n_daughters,
                        const double *parent_p4_host, const double *parent_p4_dev,
                        uint64_t ld_parent, uint64_t nevents, uint64_t seed, uint32_t stream_id,
                        uint64_t event_offset, double *p4_out_dev, uint64_t ld,
                        double *weights_dev, double *stats_dev, void *stream);

/* A sequential decay in one launch (sec. 4.2 lists sequential decays among the
 * generator's uses): the result is defined as that of two calls,
 *   hydra_phsp_generate(parent_mass, masses_host, n_daughters, NULL, NULL, 0,
 *       nevents, seed, stream_id, event_offset, p4_out_dev, ld, weights_dev,
 *       stats_dev, stream);
 *   hydra_phsp_generate(masses_host[chained], masses2_host, n2, NULL,
 *       p4_out_dev + 4 * chained * ld, ld, nevents, seed, stream_id2,
 *       event_offset, p4_out2_dev, ld2, weights2_dev, stats2_dev, stream);
 * i.e. daughter `chained` of each first-stage event (parent at rest) decays
 * into n2 daughters in its own frame, with the same event index and another
 * counter stream (stream_id2 != stream_id for independent uniforms).  Events
 * and weights of both stages are bit-identical to the two calls'; the
 * integrals agree to rounding (bit-identical when both calls run one event per
 * thread, as this launch does).  With every column on the 128-byte line grid
 * (p4_out_dev, weights_dev, p4_out2_dev, weights2_dev 128-byte aligned, ld and
 * ld2 multiples of 16) one kernel computes both stages, keeping the chained
 * daughter in registers instead of reading it back; other layouts run the two
 * calls.
 *   chained          0 .. n_daughters - 1.
 *   masses2_host, n2 the second stage's daughters, 2 <= n2 <= 4, their sum
 *                    below masses_host[chained] (EKINEMATICS otherwise).
 *   p4_out2_dev      [n2][4][ld2] doubles (device); weights2_dev [nevents];
 *   stats2_dev       NULL, or HYDRA_PHSP_STATS doubles: the second stage's integral.
 * Other arguments, layouts and errors as for hydra_phsp_generate. */
int hydra_phsp_generate_chain(double parent_mass, const double *masses_host, int n_daughters, int chained,
                              const double *masses2_host, int n2, uint64_t nevents, uint64_t seed,
                              uint32_t stream_id, uint32_t stream_id2, uint64_t event_offset,
                              double *p4_out_dev, uint64_t ld, double *weights_dev, double *stats_dev,
                              double *p4_out2_dev, uint64_t ld2, double *weights2_dev, double *stats2_dev,
                              void *stream);

/* Phase-space integral without storing events (sec. 3 lists phase-space
 * integration among the library's algorithms; sec. 4.2 the method).  The same
 * events as hydra_phsp_generate with the same (seed, stream_id, event_offset);
 * weights are Lorentz invariant, so no parent four-vector is needed.
 *   stats_dev   HYDRA_PHSP_STATS doubles (device), written asynchronously. */
int hydra_phsp_integrate_async(double parent_mass, const double *masses_host, int n_daughters,
                               uint64_t nevents, uint64_t seed, uint32_t stream_id,
                               uint64_t event_offset, double *stats_dev, void *stream);

/* Synchronous convenience form: requires nevents >= 2; returns the mean weight
 * and its standard error in host memory after synchronising `stream`. */
int hydra_phsp_integrate(double parent_mass, const double *masses_host, int n_daughters,
                         uint64_t nevents, uint64_t seed, uint32_t stream_id,
                         uint64_t event_offset, double *mean_host, double *sigma_host,
                         void *stream);

/* For callers that cannot allocate device memory: code being captured into a
 * HIP graph, tight serving loops, hosts that forbid hipMalloc.  Same arguments,
 * events, weights and stats as hydra_phsp_generate (the same kernels and the
 * same merge tree), but the block partials and merge results live in a fixed
 * device array of the library (about 24 MiB per GPU, held until the process
 * ends) instead of a per-stream workspace: the call makes no hipMalloc, hipFree
 * or other allocating call, and records no timing events.  Limit: at most
 * 2^20 blocks of 256 * ept events (ept as hydra_phsp_events_per_thread reports
 * for path 1), e.g. 2.68e8 events for n_daughters = 3, 5.37e8 for 4 and 5,
 * and 1.07e9 for 6 to 10; larger counts fail with EINVAL before any work.
 * The first call on a device performs a one-time, synchronous set-up on the
 * current device (it looks up the array's address and uploads a 4 KiB
 * trigonometric table); call it once, e.g. with nevents = 0, before capturing.
 * Every call on one GPU shares the array, so calls that overlap on one GPU
 * (other streams, other threads) race and give wrong stats; serialise them. */
int hydra_phsp_generate_noalloc(double parent_mass, const double *masses_host, int n_daughters,
                                const double *parent_p4_host, const double *parent_p4_dev,
                                uint64_t ld_parent, uint64_t nevents, uint64_t seed, uint32_t stream_id,
                                uint64_t event_offset, double *p4_out_dev, uint64_t ld,
                                double *weights_dev, double *stats_dev, void *stream);

/* ------------------------------------------------------------------------ */
/* Mixed FP32/FP64 path                                                      */
/* ------------------------------------------------------------------------ */

/* As hydra_phsp_generate (sec. 4.2), but the momentum outputs are FP32
 * (p4_out_dev is [n_daughters][4][ld] floats, half the bytes).  Every event is
 * computed in FP64 registers exactly as on the FP64 path and each component is
 * rounded once (to nearest) when stored, so the outputs are the FP64 path's
 * momenta rounded to FP32 (|dc| <= 2^-24 |c| beyond the FP64 error, for any
 * daughter masses), the weights are the FP64 path's, and so are the stats when
 * both paths run the same events per thread.  FP32 arithmetic in the boost
 * chain was rejected: a light daughter emitted against a boost of large gamma
 * loses about gamma * 2^-24 of its lab energy to an FP32 direction, beyond
 * 1e-5 for massless daughters. */
int hydra_phsp_generate_mixed(double parent_mass, const double *masses_host, int n_daughters,
                              const double *parent_p4_host, const double *parent_p4_dev,
                              uint64_t ld_parent, uint64_t nevents, uint64_t seed,
                              uint32_t stream_id, uint64_t event_offset, float *p4_out_dev,
                              uint64_t ld, double *weights_dev, double *stats_dev, void *stream);

/* ------------------------------------------------------------------------ */
/* Misc                                                                      */
/* ------------------------------------------------------------------------ */

const char *hydra_phsp_strerror(int status);
const char *hydra_phsp_last_error(void);
int hydra_phsp_abi_version(void);
/* Host-side self-test of the in-register sorting networks (0-1 principle over
 * every network the kernels use); returns HYDRA_PHSP_OK when all sort. */
int hydra_phsp_selftest_sortnet(void);
/* Events per thread of the single-channel kernels, per path: path 0 =
 * integrate-only, 1 = FP64 generate, 2 = mixed generate; ept in {1, 2, 4}, or 0
 * for the library default.  Defaults with columns on the 128-byte line grid:
 * integrate 4; FP64 generate 2, 1, 2, 2, 4, 4, 4, 4, 4 and mixed generate 2,
 * 4, 4, 4, 4, 4, 4, 4, 4 for N = 2..10; 1 with per-event parents for N <= 3.
 * Columns off the line grid (the staged kernel) have their own: FP64 2, 4, 2,
 * 1, 1, 1, 1, 1, 1 and mixed 4, 4, 2, 1, 1, 1, 1, 1, 1 for N = 2..10 (any
 * parent mode).  One launch covers at most
 * (2^32 - 1) / 256 * ept events; larger counts are rejected with EINVAL.
 * Process-wide; changes the launch shape only (events are bit-identical for
 * every value; integrals agree to rounding). */
int hydra_phsp_set_events_per_thread(int path, int ept);
/* The events per thread the next single-channel launch on `path` would use for
 * n_daughters, after any override.  flags: bit 0 (1) with per-event parent
 * four-vectors, bit 1 (2) with columns off the 128-byte line grid.  EINVAL for
 * a bad path, n_daughters or flags. */
#define HYDRA_PHSP_EPT_PER_EVENT_PARENTS 1
#define HYDRA_PHSP_EPT_OFF_LINE_GRID 2
int hydra_phsp_events_per_thread(int path, int n_daughters, int flags);

/* Statistics of two disjoint sets of events merged into those of their union
 * (host records of HYDRA_PHSP_STATS doubles: n, mean, M2, sigma), with the
 * pairwise update of Chan, Golub and LeVeque that the kernels' reduction uses:
 * n = na + nb, mean = ma + (mb - ma) nb / n, M2 = M2a + M2b + (mb - ma)^2 na nb / n,
 * sigma recomputed.  This is how the integral of a job taken in pieces (a
 * resumed job, or shards on several devices, each an event_offset range of the
 * same seed and stream id) is assembled: the state of such a job is (seed,
 * stream id, next event_offset, stats so far), and merging the pieces left to
 * right in event order gives a deterministic result, equal to the single
 * call's up to rounding (sec. 3 of arXiv:1711.05683: the Monte Carlo estimate
 * is the mean weight, its error the standard error of the mean).  out_host may
 * alias a_host or b_host.  EINVAL for a NULL pointer, a negative,
 * non-integral or non-finite n, or a non-finite mean or M2, or a negative M2. */
int hydra_phsp_stats_merge(const double *a_host, const double *b_host, double *out_host);

/* Kernel timing for benchmarks: while enabled, every launch of the main
 * phase-space kernel is bracketed by HIP events recorded on the caller's
 * stream.  hydra_phsp_timing_read synchronises those events and returns the
 * summed kernel time (ms) and the number of launches since the last reset. */
int hydra_phsp_timing_enable(int on);
int hydra_phsp_timing_read(double *total_ms_host, uint64_t *launches_host);
int hydra_phsp_timing_reset(void);
/* Free every cached device workspace of the library (single-channel block
 * partials, the tables of the last batch per stream, the unweighting and VEGAS
 * workspaces), after synchronising the device.  Not to be called while another
 * thread is inside a library call; later calls allocate afresh. */
int hydra_phsp_release(void);

#ifdef __cplusplus
}
#endif

#endif /* HYDRA_PHSP_H */

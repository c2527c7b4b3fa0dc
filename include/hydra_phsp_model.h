/*
 * hydra_phsp_model.h -- evaluation of a model over phase space.
 *
 * Sec. 4.2 of arXiv:1711.05683 lists the evaluation of a model over the
 * generated phase space among the generator's uses.  Here the model is a
 * product of relativistic Breit-Wigner intensities in pair invariant masses,
 *   |A|^2 = prod_k 1 / ((M_k^2 - s_k)^2 + M_k^2 G_k^2),
 *   s_k = (p_i + p_j)^2 for the daughters (i, j) of factor k,
 * evaluated on each generated event (parent at rest) and integrated with the
 * event weights: the mean of w |A|^2 is the integral of |A|^2 over phase space.
 * With no factor |A|^2 = 1 and the result is the phase-space volume.
 * Conventions, ownership and error codes are those of hydra_phsp.h.
 */
#ifndef HYDRA_PHSP_MODEL_H
#define HYDRA_PHSP_MODEL_H

#include <stdint.h>

#include "hydra_phsp.h"

#ifdef __cplusplus
extern "C" {
#endif

#define HYDRA_PHSP_MAX_BW 4

typedef struct hydra_phsp_breit_wigner {
    int32_t i, j;  /* daughters of the pair, 0 <= i < j < n_daughters */
    double mass;   /* M_k > 0 */
    double width;  /* G_k > 0 */
} hydra_phsp_breit_wigner;

/* Integrate the model over `nevents` events (global indices event_offset ..),
 * asynchronous on `stream`.
 *   resonances_host  n_resonances (0 .. HYDRA_PHSP_MAX_BW) factors (host).
 *   values_dev       NULL, or [nevents] doubles (device): w |A|^2 per event.
 *   stats_dev        HYDRA_PHSP_STATS doubles (device): n, mean (the integral),
 *                    M2, sigma of the per-event values.
 * The events, weights and draws are those of hydra_phsp_generate with the same
 * (masses, seed, stream_id, event_offset); with no factor the stats equal those
 * of hydra_phsp_integrate_async with four events per thread.  EINVAL for a bad
 * factor (pair out of range or not i < j, mass or width not finite and > 0),
 * a NULL stats_dev or misaligned pointers; EKINEMATICS as for generate. */
int hydra_phsp_integrate_model(double parent_mass, const double *masses_host, int n_daughters,
                               const hydra_phsp_breit_wigner *resonances_host, int n_resonances,
                               uint64_t nevents, uint64_t seed, uint32_t stream_id, uint64_t event_offset,
                               double *values_dev, double *stats_dev, void *stream);

/* ---------------------------------------------------------------------------
 * User intensities, compiled at run time.  Hydra evaluates user code passed as
 * functors with parameters (sec. 3.1 of arXiv:1711.05683); here the user
 * passes HIP device source that defines
 *
 *   __device__ double hydra_phsp_user_intensity(const double *e,
 *       const double *px, const double *py, const double *pz,
 *       const double *par);
 *
 * receiving the N daughters' four-momenta (E, px, py, pz)[0..N-1] in the
 * parent's rest frame, in caller order, and the parameters par[0..15] (the
 * n_params given at evaluation, then zeros), and returning |A|^2 >= 0.  The
 * macro HYDRA_PHSP_N holds N; the source may define helpers of its own (names
 * starting with hphsp or hydra_phsp_user_model are the library's).  The
 * library compiles the source with hiprtc for gfx950 (-O3, no floating-point
 * contraction) together with its own kernel headers into one kernel that
 * generates each event in registers and applies the function to it (inlined),
 * so a model runs at the speed of the built-in Breit-Wigner product.
 * ------------------------------------------------------------------------- */
typedef struct hydra_phsp_user_model hydra_phsp_user_model;

/* Compile `source_host` (NUL-terminated) for events of n_daughters (2..10)
 * daughters; *model_out receives the model (owned by the caller: release it
 * with hydra_phsp_user_model_destroy).  Compilation needs no GPU; the code
 * object is loaded on each device at its first evaluation there.  EINVAL for a
 * NULL argument, n_daughters out of range, or a source that does not compile
 * (the compiler's log, up to 8 KiB, is in hydra_phsp_last_error); EDEVICE when
 * hiprtc itself fails.  Calls on one model may come from several threads;
 * create and destroy must not overlap its evaluations. */
int hydra_phsp_user_model_create(const char *source_host, int n_daughters, hydra_phsp_user_model **model_out);

/* Waits for the devices the model was loaded on, unloads it and frees it. */
int hydra_phsp_user_model_destroy(hydra_phsp_user_model *model);

/* The model's number of daughters (or EINVAL for NULL). */
int hydra_phsp_user_model_daughters(const hydra_phsp_user_model *model);

/* Integrate the user's intensity over `nevents` events, asynchronous on
 * `stream`: as hydra_phsp_integrate_model, with masses_host holding the
 * model's N daughter masses and params_host n_params (0..16) doubles (host;
 * NULL when n_params is 0).  values_dev (NULL or [nevents]) receives
 * w |A|^2 per event, stats_dev (n, mean, M2, sigma) of those values; with
 * |A|^2 = 1 the stats are those of hydra_phsp_integrate_async with four events
 * per thread, and a source that computes the built-in Breit-Wigner product the
 * same way gives the same values as hydra_phsp_integrate_model.  EINVAL for a
 * NULL model or stats_dev, n_params out of range, NULL params with n_params >
 * 0, misaligned pointers; EKINEMATICS as for generate; EDEVICE when the code
 * object does not load. */
int hydra_phsp_integrate_user_model(hydra_phsp_user_model *model, double parent_mass, const double *masses_host,
                                    const double *params_host, int n_params, uint64_t nevents, uint64_t seed,
                                    uint32_t stream_id, uint64_t event_offset, double *values_dev,
                                    double *stats_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HYDRA_PHSP_MODEL_H */

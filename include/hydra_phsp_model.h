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

#ifdef __cplusplus
}
#endif

#endif /* HYDRA_PHSP_MODEL_H */

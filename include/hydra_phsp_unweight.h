/*
 * hydra_phsp_unweight.h -- unweighted phase-space samples.
 *
 * Sec. 4.2 of arXiv:1711.05683 lists unweighted samples beside the weighted
 * ones.  This is the hit-or-miss method: trial event g (the weighted event
 * hydra_phsp_generate produces for the same seed, stream_id and global index
 * g) is kept when v_g * w_max < w_g, where w_g is its weight and v_g its
 * acceptance uniform: words 0 and 1 of Philox4x32-10 call j = ceil((3N-4)/2) of
 * the event's counter stream (the first call its own uniforms do not use),
 * converted like every other uniform, (2x+1) 2^-53 with x the top 52 bits.
 * Kept events therefore follow the phase-space density with unit weight.
 * Conventions, layouts, ownership and error codes are those of hydra_phsp.h.
 */
#ifndef HYDRA_PHSP_UNWEIGHT_H
#define HYDRA_PHSP_UNWEIGHT_H

#include <stdint.h>

#include "hydra_phsp.h"
#include "hydra_phsp_model.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Hit-or-miss sample from ntrials weighted trials (global indices event_offset
 * .. event_offset + ntrials - 1).  Asynchronous on `stream`.
 *
 *   parent_mass, masses_host, n_daughters, parent_p4_host, seed, stream_id,
 *   event_offset  as for hydra_phsp_generate (parent at rest or one broadcast
 *                 parent four-vector).
 *   w_max         > 0: the bound (trials with a larger weight are always kept
 *                 and counted in counts_dev[1]); 0: the largest weight among
 *                 the trials, found by an extra pass over them.
 *   p4_out_dev    NULL, or the kept events in trial order, SoA
 *                 [n_daughters][4][ld] doubles (device).
 *   ld            capacity in events when p4_out_dev or index_out_dev is given
 *                 (>= 1); kept events past the capacity are counted but not
 *                 written.
 *   index_out_dev NULL, or [ld] uint64 (device): the global index of each kept
 *                 event, increasing.
 *   counts_dev    required, 2 uint64 (device): [0] number kept (all of them,
 *                 also past the capacity), [1] number of trials whose weight
 *                 exceeded w_max.
 *   w_max_dev     NULL, or 1 double (device) receiving the bound applied.
 *
 * With both outputs NULL only the counts are produced (no kinematics are
 * computed).  EINVAL for a negative or non-finite w_max, a NULL counts_dev, a
 * zero capacity with outputs, misaligned pointers or ntrials beyond one
 * launch ((2^32 - 1) / 256 * 1024 trials); EKINEMATICS as for generate. */
int hydra_phsp_generate_unweighted(double parent_mass, const double *masses_host, int n_daughters,
                                   const double *parent_p4_host, uint64_t ntrials, uint64_t seed,
                                   uint32_t stream_id, uint64_t event_offset, double w_max,
                                   double *p4_out_dev, uint64_t ld, uint64_t *index_out_dev,
                                   uint64_t *counts_dev, double *w_max_dev, void *stream);

/* Pipeline depth of the unweighted calls that store events, process-wide: the
 * trials are cut into at most `chunks` chunks (each at least 262144 trials), and
 * one launch stores the kept events of a chunk while it computes the keep
 * decisions of the next.  1 runs the passes one after the other; 0 restores the
 * defaults: 4 for acceptance against the weight alone, 1 for Breit-Wigner
 * models (their kept fraction is usually small, so there is little store work
 * to overlap and each chunk costs a scan and a launch tail).  User models
 * (compiled at run time) always take one chunk.  The results are the same for
 * every value.  EINVAL outside [0, 16]. */
int hydra_phsp_set_unweight_chunks(int chunks);

/* Unweighted samples of a model (sec. 4.2 lists weighted and unweighted
 * samples and model evaluation together): trial event g is kept when
 * v_g * w_max < w_g |A|^2(g), with |A|^2 the product of Breit-Wigner factors of
 * hydra_phsp_integrate_model, the parent at rest and v_g the acceptance uniform
 * above.  Kept events then follow |A|^2 times the phase-space density.  The
 * trials, draws, outputs, counts and bound are those of
 * hydra_phsp_generate_unweighted with w_g replaced by w_g |A|^2(g) (w_max = 0:
 * the largest w |A|^2 among the trials; counts_dev[1] the trials above the
 * bound); with no factor the result is that of hydra_phsp_generate_unweighted.
 * With w_max = 0 and at most 2^28 trials the library keeps each trial's value
 * between the maximum and the count passes instead of computing it twice
 * (8 bytes per trial in its per-stream workspace, kept until
 * hydra_phsp_release; the results are the same either way).
 * EINVAL for a bad factor (as for hydra_phsp_integrate_model) and as above. */
int hydra_phsp_generate_unweighted_model(double parent_mass, const double *masses_host, int n_daughters,
                                         const hydra_phsp_breit_wigner *resonances_host, int n_resonances,
                                         uint64_t ntrials, uint64_t seed, uint32_t stream_id,
                                         uint64_t event_offset, double w_max, double *p4_out_dev, uint64_t ld,
                                         uint64_t *index_out_dev, uint64_t *counts_dev, double *w_max_dev,
                                         void *stream);

/* The same with a user intensity compiled by hydra_phsp_user_model_create
 * (n_daughters is the model's): trial g is kept when
 * v_g * w_max < w_g * hydra_phsp_user_intensity(event g, params), with the
 * n_params (0 .. HYDRA_PHSP_USER_PARAMS) params_host values, then zeros.  The
 * first call on a device loads the model's code there.  EINVAL for a NULL
 * model, n_params out of range or params_host NULL with n_params > 0, and as
 * above.  Trial values are kept between passes as for the Breit-Wigner model. */
int hydra_phsp_generate_unweighted_user_model(hydra_phsp_user_model *model, double parent_mass,
                                              const double *masses_host, const double *params_host, int n_params,
                                              uint64_t ntrials, uint64_t seed, uint32_t stream_id,
                                              uint64_t event_offset, double w_max, double *p4_out_dev, uint64_t ld,
                                              uint64_t *index_out_dev, uint64_t *counts_dev, double *w_max_dev,
                                              void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HYDRA_PHSP_UNWEIGHT_H */

/*
 * hydra_phsp_vegas.h -- VEGAS importance-sampling integration and plain Monte
 * Carlo (a second workload on the generator's counter-based random numbers and
 * fused reduction).
 *
 * The paper (arXiv:1711.05683, sec. 3 and 4.1) lists plain and self-adaptive
 * importance-sampling Monte Carlo integration and benchmarks VEGAS (Lepage,
 * J. Comput. Phys. 27 (1978) 192) on a 10-dimensional Gaussian; it follows the
 * structure of the GSL implementation and parallelises the integrand
 * evaluations and accumulations of each iteration.  Here:
 *
 *   integrand  f(x) = prod_d exp(-(x_d - mean_d)^2 / (2 sigma_d^2)) /
 *              (sigma_d sqrt(2 pi)) over the box prod_d [lo_d, hi_d];
 *   grid       per dimension K bins, edges g[0] = 0 < ... < g[K] = 1 in unit
 *              coordinates, stored [dim][K+1];
 *   sample i   of iteration t: uniform d is uniform d of the counter stream
 *              (i lo, i hi, call, t) under the seed (two Philox4x32-10 words per
 *              uniform, (2x+1) 2^-53); z = K u, b = floor(z),
 *              y = g[b] + (z - b)(g[b+1] - g[b]), x_d = lo_d + y (hi_d - lo_d);
 *              value = f(x) prod_d K (g[b+1] - g[b]) (hi_d - lo_d);
 *   estimate   the mean value and its standard error (HYDRA_PHSP_STATS layout);
 *   histogram  value^2 summed per (dimension, bin), [dim][K];
 *   refinement per dimension: the histogram smoothed with its neighbours
 *              ((h0+h1)/2, (h[k-1]+h[k]+h[k+1])/3, (h[K-2]+h[K-1])/2), each bin's
 *              damped importance ((1 - 1/R)/ln R)^alpha with R = (smoothed
 *              total)/(smoothed bin), and the old grid re-cut into K pieces of
 *              equal importance (a bin's importance spread evenly over it).
 *
 * Plain Monte Carlo is one iteration on the uniform grid (g[k] = k/K).
 */
#ifndef HYDRA_PHSP_VEGAS_H
#define HYDRA_PHSP_VEGAS_H

#include <stdint.h>

#include "hydra_phsp.h"

#ifdef __cplusplus
extern "C" {
#endif

#define HYDRA_PHSP_VEGAS_DMAX 16
#define HYDRA_PHSP_VEGAS_KMAX 128

typedef struct hydra_phsp_gauss_box {
    int32_t dim; /* 1 .. HYDRA_PHSP_VEGAS_DMAX */
    int32_t reserved;
    double lo[HYDRA_PHSP_VEGAS_DMAX], hi[HYDRA_PHSP_VEGAS_DMAX];      /* box, hi > lo */
    double mean[HYDRA_PHSP_VEGAS_DMAX], sigma[HYDRA_PHSP_VEGAS_DMAX]; /* sigma > 0 */
} hydra_phsp_gauss_box;

/* One iteration, asynchronous on `stream`: `calls` (>= 2) samples on grid_dev
 * ([dim][bins+1] doubles, device; 2 <= bins <= HYDRA_PHSP_VEGAS_KMAX);
 * stats_dev (HYDRA_PHSP_STATS doubles) receives n, mean (the estimate), M2,
 * sigma; hist_dev (NULL or [dim][bins] doubles) the refinement histogram;
 * values_dev (NULL or [calls] doubles) each sample's value. */
int hydra_phsp_vegas_iteration(const hydra_phsp_gauss_box *f, int bins, const double *grid_dev, uint64_t calls,
                               uint64_t seed, uint32_t iteration, double *stats_dev, double *hist_dev,
                               double *values_dev, void *stream);

/* Refine a host grid ([dim][bins+1]) in place from a host histogram ([dim][bins])
 * with damping exponent alpha >= 0 (1.5 is customary). */
int hydra_phsp_vegas_refine(int dim, int bins, double *grid_host, const double *hist_host, double alpha);

/* The whole integration, synchronous: `warmup` iterations that only adapt the
 * grid, then `iterations` that also estimate (iteration t uses counter word 3 =
 * t); each iteration is followed by a refinement.  result / error: the
 * inverse-variance weighted mean of the estimating iterations and its error;
 * chi2_dof: their chi^2 per degree of freedom.  grid_host: NULL (start uniform)
 * or [dim][bins+1] doubles, the starting grid on input and the final grid on
 * output. */
int hydra_phsp_vegas(const hydra_phsp_gauss_box *f, int bins, uint64_t calls, int warmup, int iterations,
                     double alpha, uint64_t seed, double *grid_host, double *result, double *error,
                     double *chi2_dof, void *stream);

/* ---------------------------------------------------------------------------
 * User integrands, compiled at run time (the paper's integrators take user
 * functors, sec. 3.1; its VEGAS benchmark is the Gaussian above).  The user
 * passes HIP device source that defines
 *
 *   __device__ double hydra_phsp_user_integrand(const double *x,
 *                                               const double *par);
 *
 * receiving a sample's coordinates x[0..dim-1] in the box and the parameters
 * par[0..15] (the n_params given, then zeros); the macro HYDRA_PHSP_DIM holds
 * dim.  The library compiles it with hiprtc for gfx950 (-O3, no floating-point
 * contraction) into the VEGAS kernel with the function inlined in place of the
 * Gaussian product: the samples, grid, histogram, reduction and refinement are
 * those described above, with value = f(x) times the Jacobian.
 * ------------------------------------------------------------------------- */
typedef struct hydra_phsp_user_integrand hydra_phsp_user_integrand;

/* Compile `source_host` (NUL-terminated) for dim (1..16) dimensions;
 * *integrand_out receives the integrand (release it with
 * hydra_phsp_user_integrand_destroy).  Compilation needs no GPU; the code
 * object is loaded on each device at its first use there.  EINVAL for a NULL
 * argument, dim out of range, or a source that does not compile (the
 * compiler's log, up to 8 KiB, is in hydra_phsp_last_error); EDEVICE when
 * hiprtc itself fails. */
int hydra_phsp_user_integrand_create(const char *source_host, int dim, hydra_phsp_user_integrand **integrand_out);

/* Waits for the devices the integrand was loaded on, unloads it and frees it. */
int hydra_phsp_user_integrand_destroy(hydra_phsp_user_integrand *integrand);

/* As hydra_phsp_vegas_iteration for the user's integrand over the box
 * [lo_host[d], hi_host[d]] (host, dim doubles each, hi > lo) with n_params
 * (0..16) parameters params_host (host; NULL when n_params is 0).  EINVAL also
 * for a NULL integrand or box, a bad box edge or n_params out of range. */
int hydra_phsp_vegas_user_iteration(hydra_phsp_user_integrand *f, const double *lo_host, const double *hi_host,
                                    const double *params_host, int n_params, int bins, const double *grid_dev,
                                    uint64_t calls, uint64_t seed, uint32_t iteration, double *stats_dev,
                                    double *hist_dev, double *values_dev, void *stream);

/* As hydra_phsp_vegas (the whole integration, synchronous) for the user's
 * integrand over the box with the given parameters. */
int hydra_phsp_vegas_user(hydra_phsp_user_integrand *f, const double *lo_host, const double *hi_host,
                          const double *params_host, int n_params, int bins, uint64_t calls, int warmup,
                          int iterations, double alpha, uint64_t seed, double *grid_host, double *result,
                          double *error, double *chi2_dof, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HYDRA_PHSP_VEGAS_H */

/*
 * hydra_phsp_probe.h -- measurement probes for the two ceilings of the
 * generator.
 *
 * Sec. 4.2 of arXiv:1711.05683 reports the generator's time against the sample
 * size (figure "fig:phsp") and nothing about what bounds it.  Per event the
 * generator writes 4N + 1 doubles and makes ceil((3N - 4) / 2) calls of the
 * counter-based generator, so two rates bound it on a given device: the
 * streaming-write rate of its structure-of-arrays output, and the rate of the
 * Philox4x32-10 calls.  These probes measure each alone, with the generator's
 * own launch shape, store pattern and Philox code, and nothing else.
 *
 * Both are asynchronous on `stream` (a hipStream_t; NULL = the null stream),
 * validate every argument before enqueueing anything, and return the status
 * codes of hydra_phsp.h.  They allocate nothing.
 */
#ifndef HYDRA_PHSP_PROBE_H
#define HYDRA_PHSP_PROBE_H

#include <stdint.h>

#include "hydra_phsp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Events one block of the Philox probe covers: fold_dev holds
 * ceil(nevents / HYDRA_PHSP_PROBE_SPAN) words. */
#define HYDRA_PHSP_PROBE_SPAN 1024

/* Streaming-write probe: out_dev[c * ld + e] = c for every column
 * c < n_columns and event e < nevents, and weights_dev[e] = -1, with the
 * generator's stores (block of 256 lanes covering 256 * events_per_thread
 * consecutive events, one event per lane per step, non-temporal 8-byte stores
 * of every column of the event in column order, then its weight).  For the
 * pattern of an N-body generate call pass n_columns = 4N and the same ld,
 * buffers and events per thread.
 *   out_dev             [n_columns][ld] doubles (device), 8-byte aligned.
 *   ld                  >= nevents.
 *   n_columns           1 .. 4 * HYDRA_PHSP_NMAX.
 *   weights_dev         [nevents] doubles (device), 8-byte aligned.
 *   events_per_thread   1, 2 or 4.
 * nevents = 0 enqueues nothing.  EINVAL for a NULL pointer, ld < nevents, a
 * count out of range, or a grid above 2^32 - 1 threads. */
int hydra_phsp_probe_write(double *out_dev, uint64_t ld, int n_columns, double *weights_dev,
                           uint64_t nevents, int events_per_thread, void *stream);

/* Philox probe: for every event e < nevents, calls j = 0 .. calls_per_event-1
 * of Philox4x32-10 with key (seed lo, seed hi) and counter
 * (e lo, e hi, j, stream_id) -- the draws of the generator's event e -- and the
 * exclusive or of all four words of every call of the HYDRA_PHSP_PROBE_SPAN
 * events of block b is written to fold_dev[b].
 *   calls_per_event   1 .. 16.
 *   fold_dev          ceil(nevents / HYDRA_PHSP_PROBE_SPAN) words (device),
 *                     4-byte aligned.
 * nevents = 0 enqueues nothing.  EINVAL for a NULL pointer or a count out of
 * range. */
int hydra_phsp_probe_philox(uint64_t nevents, int calls_per_event, uint64_t seed, uint32_t stream_id,
                            uint32_t *fold_dev, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HYDRA_PHSP_PROBE_H */

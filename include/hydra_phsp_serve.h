/*
 * hydra_phsp_serve.h -- continuous-batching request server for phase-space
 * generation and integration (the generator of arXiv:1711.05683 sec. 4.2
 * serving many independent requests on one GPU).
 *
 * Requests (one decay channel each, generate or integrate-only) are queued by
 * submit; each scheduling step retires finished work, admits queued requests
 * while the server's HBM budget and active-slot limit allow, and enqueues one
 * "tick": a persistent-kernel launch over the tiles of every active request
 * (oldest first, up to the per-tick event cap), followed by the merges of the
 * requests whose last tiles it holds.  Ticks run back to back on the server's
 * stream while the host prepares the next, so requests that arrive while
 * others are on the GPU join the next tick.  Random-number state (the event
 * counters) and partial sums stay on the device between ticks.
 *
 * A request's events, weights and integral depend only on the request itself
 * (tiles of 256 events with the request's own seed/stream counters, a merge
 * tree fixed by its event count), so every result is bit-identical whether the
 * request ran alone or in any mix.  Conventions are those of hydra_phsp.h.
 */
#ifndef HYDRA_PHSP_SERVE_H
#define HYDRA_PHSP_SERVE_H

#include <stdint.h>

#include "hydra_phsp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hydra_phsp_server hydra_phsp_server;

typedef struct hydra_phsp_request {
    double parent_mass;
    double masses[HYDRA_PHSP_NMAX];
    int32_t n_daughters;
    int32_t integrate_only; /* 1: no event storage, integral only */
    uint64_t nevents;       /* >= 1 */
    uint64_t seed;
    uint32_t stream_id;
    uint32_t reserved;
} hydra_phsp_request;

typedef struct hydra_phsp_result {
    int32_t status;      /* HYDRA_PHSP_OK once finished */
    int32_t n_daughters;
    uint64_t nevents;
    double mean, sigma;  /* integral of the request's weights */
    double *p4_dev;      /* server-owned SoA [n][4][nevents]; NULL if integrate-only */
    double *weights_dev; /* server-owned [nevents]; NULL if integrate-only */
    double submit_s, admit_s, done_s; /* host monotonic clock, seconds */
} hydra_phsp_result;

/* Create a server on the current device.  hbm_budget_bytes bounds the device
 * memory held by admitted requests (outputs + partial sums; the arena is
 * allocated once); max_events_per_tick bounds one tick (0 = 2^22);
 * max_active bounds the requests admitted at once (0 = 1024). */
int hydra_phsp_server_create(uint64_t hbm_budget_bytes, uint64_t max_events_per_tick, int max_active,
                             hydra_phsp_server **server_out);
/* Queue a request (thread-safe).  An invalid request, or one that can never
 * fit the budget, fails here with its own status and leaves the rest intact. */
int hydra_phsp_server_submit(hydra_phsp_server *server, const hydra_phsp_request *req,
                             uint64_t *id_out);
/* One scheduling step (retire, admit, enqueue a tick).  Returns the number of
 * requests queued or in flight (>= 0), or a negative status on a device error.
 * Steps must be called from one thread at a time. */
int hydra_phsp_server_step(hydra_phsp_server *server);
/* Up to max ids of requests finished since the last call (host array). */
int hydra_phsp_server_completed(hydra_phsp_server *server, uint64_t *ids_out, int max);
/* A request's result: OK when finished, EAGAIN while queued or running,
 * ENOTFOUND for an unknown or released id. */
int hydra_phsp_server_poll(hydra_phsp_server *server, uint64_t id, hydra_phsp_result *res);
/* Return a finished request's device memory to the budget and forget it. */
int hydra_phsp_server_release(hydra_phsp_server *server, uint64_t id);
/* Drain: step until every submitted request has finished. */
int hydra_phsp_server_drain(hydra_phsp_server *server);

/* Native replay of an arrival trace in real time (a load generator for
 * benchmarks): request i is submitted at arrival_s[i] seconds after the start;
 * the loop steps the server, releases results as they finish and writes each
 * request's latency (finish - arrival, seconds) to latency_s_out[i] (host).
 * wall_s_out receives the total wall time; peak_bytes_out the largest arena
 * use.  Requests that fail at submit get latency -1. */
int hydra_phsp_server_replay(hydra_phsp_server *server, const hydra_phsp_request *reqs,
                             const double *arrival_s, int n, double *latency_s_out,
                             double *wall_s_out, uint64_t *peak_bytes_out);

/* Counters: bytes in use, peak bytes, ticks launched, requests finished. */
int hydra_phsp_server_stats(const hydra_phsp_server *server, uint64_t *bytes_in_use,
                            uint64_t *peak_bytes, uint64_t *ticks, uint64_t *finished);

/* Admission counters since creation (all host-side). */
typedef struct hydra_phsp_server_counters {
    uint64_t bytes_in_use, peak_bytes, ticks, finished;
    uint64_t budget_stalls;  /* steps that left the queue's head waiting for HBM budget */
    uint64_t active_stalls;  /* steps that left it waiting for an active slot */
    double queue_wait_max_s; /* longest submit -> admit wait of a finished request */
    double queue_wait_sum_s; /* summed submit -> admit waits of finished requests */
} hydra_phsp_server_counters;
int hydra_phsp_server_counters_get(const hydra_phsp_server *server, hydra_phsp_server_counters *out);
/* Wait for all outstanding device work, then free everything. */
int hydra_phsp_server_destroy(hydra_phsp_server *server);

#ifdef __cplusplus
}
#endif

#endif /* HYDRA_PHSP_SERVE_H */

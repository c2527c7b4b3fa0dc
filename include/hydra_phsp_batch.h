/*
 * hydra_phsp_batch.h -- batched multi-channel phase-space generation.
 *
 * Many decay channels of uneven daughter count and event count run in one
 * submission: one kernel launch per (daughter count, mode) class present, each
 * specialised like the single-channel kernel for that class (the phase-space
 * generator of arXiv:1711.05683 sec. 4.2, applied to many (M, masses) pairs at
 * once).  Conventions,
 * layouts, ownership and error codes are those of hydra_phsp.h.
 */
#ifndef HYDRA_PHSP_BATCH_H
#define HYDRA_PHSP_BATCH_H

#include <stdint.h>

#include "hydra_phsp.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One decay channel: the arguments of one hydra_phsp_generate call with the
 * parent at rest.  p4_out_dev and weights_dev both NULL means integrate-only.
 * stats_dev (HYDRA_PHSP_STATS doubles, device) is required.  Each channel's
 * events and weights are bit-identical to a single-channel call with the same
 * (masses, seed, stream_id, event_offset); its stats are bit-identical too when
 * the single-channel call ran with the same events per thread (always so with
 * tuning ept 0, see hydra_phsp_tuning), and agree to rounding otherwise. */
typedef struct hydra_phsp_channel {
    double parent_mass;
    double masses[HYDRA_PHSP_NMAX];
    int32_t n_daughters;
    uint32_t stream_id;
    uint64_t nevents;
    uint64_t seed;
    uint64_t event_offset;
    double *p4_out_dev;  /* [n][4][ld] or NULL */
    uint64_t ld;
    double *weights_dev; /* [nevents] or NULL */
    double *stats_dev;   /* HYDRA_PHSP_STATS doubles */
} hydra_phsp_channel;

/* Launch shape of the batched kernels (blocks of 256 threads):
 *   ept          events per thread: 1, 2 or 4 for every class (a tile is
 *                256*ept events), or 0: per class, what a single-channel call
 *                of that N, mode and layout (columns on or off the 128-byte
 *                line grid) would use (hydra_phsp_events_per_thread), so every
 *                channel's tiles are the blocks of that call on its buffers;
 *   grid_per_cu  persistent blocks per compute unit, 1 .. 64 (schedules 0, 1,
 *                4, 5);
 *   schedule     one launch per (N, mode, layout) class:
 *                0: persistent grid, static stride over the tiles;
 *                1: persistent grid, blocks claim tiles in order from a
 *                   device counter;
 *                2: one block per tile (grid = tile count, grid_per_cu is
 *                   ignored), so the hardware dispatches tiles in order;
 *                one launch over the tiles of every channel, heaviest tiles
 *                first (a tile's events times the columns it writes, or times
 *                N for integrate-only channels), in one kernel that switches on
 *                each tile's N:
 *                3: one block per tile;
 *                4: persistent grid, static stride;
 *                5: persistent grid, blocks claim tiles from a device counter;
 *                these take ept 0 (every N and mode at the single-channel
 *                default for columns on the line grid; the compiled defaults
 *                apply even when hydra_phsp_set_events_per_thread has
 *                overridden them, so events, weights and stats are those of
 *                single-channel calls with default settings) or ept 1 (one
 *                event per thread), run on one stream, and need every
 *                generating channel's columns on the 128-byte line grid (else
 *                EINVAL);
 *   streams      0 or 1: the class kernels run one after another on the
 *                caller's stream; 2 .. HYDRA_PHSP_MAX_CLASS_STREAMS: they are
 *                spread over that many streams (the caller's and the plan's
 *                own, forked from and joined back into the caller's stream
 *                with events, largest classes first onto the least loaded
 *                stream), so kernels of different classes -- memory-bound
 *                small N beside arithmetic-bound large N -- can run at the
 *                same time.  Results do not depend on it (classes write
 *                disjoint outputs and partials; the merges follow the join).
 * A zero grid_per_cu selects the library default: 8 for schedules 0 and 1, 4
 * for schedules 4 and 5 (whose kernel fits four 256-thread blocks on a compute
 * unit). */
#define HYDRA_PHSP_MAX_CLASS_STREAMS 4
typedef struct hydra_phsp_tuning {
    int32_t ept;
    int32_t grid_per_cu;
    int32_t schedule;
    int32_t streams;
} hydra_phsp_tuning;

/* Enqueue one batch on `stream`: validates every channel (no work is enqueued
 * if any channel is invalid; *bad_channel_out, when not NULL, receives the
 * index of the first bad one), uploads the tile table and launches the
 * class kernels and the per-channel merges.  The device tables stay alive
 * until the next hydra_phsp_batch_run on the same stream, which first waits
 * for this one.  tuning may be NULL. */
int hydra_phsp_batch_run(const hydra_phsp_channel *channels, int n_channels,
                         const hydra_phsp_tuning *tuning, void *stream, int *bad_channel_out);

/* A reusable batch: tables are built and uploaded once and the launch sequence
 * (class kernels + per-channel merges) is captured into a HIP graph that
 * hydra_phsp_plan_launch replays on any stream.  The channels, including their
 * device pointers, are fixed at creation.  One plan's launches must not
 * overlap each other. */
typedef struct hydra_phsp_plan hydra_phsp_plan;
int hydra_phsp_plan_create(const hydra_phsp_channel *channels, int n_channels,
                           const hydra_phsp_tuning *tuning, hydra_phsp_plan **plan_out);
int hydra_phsp_plan_launch(hydra_phsp_plan *plan, void *stream);
/* Waits for the plan's outstanding launches, then frees it. */
int hydra_phsp_plan_destroy(hydra_phsp_plan *plan);
/* Number of tiles and the largest class grid of a plan (host). */
int hydra_phsp_plan_info(const hydra_phsp_plan *plan, uint64_t *ntiles_out, uint64_t *grid_out);

/* Autotuner: times the batch (kernels and merges) over schedule
 * {static, dynamic} x events per thread {per class, 1, 2, 4} x blocks per
 * compute unit {1, 2, 4, 8, 16}, plus one block per tile x events per thread,
 * plus the single launches (when every column is on the line grid: schedules
 * 3, 4 and 5 at events per thread {0, 1}, 4 and 5 at 1, 2 and 4 blocks per
 * compute unit), on one stream, then the best per-class shape on 2 .. HYDRA_PHSP_MAX_CLASS_STREAMS
 * streams -- two warm-up
 * runs and five timed runs per shape, overwriting the batch's outputs -- and
 * returns the shape with the fastest run and that run's time in ms.  Results
 * are cached per device and batch shape class (channel count, largest N,
 * integrate-only and off-line-grid channel counts, total events to a quarter
 * octave) for the life of the process; a cached answer is returned without
 * running.  When the environment variable HYDRA_PHSP_TUNE_CACHE names a file,
 * answers are also looked up in it (after the process's own cache) and new ones
 * appended to it, one text line per device architecture and compute-unit
 * count and shape class, so later processes skip the sweep; a missing or
 * unwritable file is ignored. */
int hydra_phsp_autotune(const hydra_phsp_channel *channels, int n_channels, void *stream,
                        hydra_phsp_tuning *best_out, double *best_ms_out);

#ifdef __cplusplus
}
#endif

#endif /* HYDRA_PHSP_BATCH_H */

/*
 * abi_host_driver.c -- the host side of the C ABI under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Every device-facing call below is given an
 * argument that validation must reject (fake device pointers such as 0x100 are
 * never dereferenced), so the run touches no GPU; the host-only routines
 * (error strings, the sorting-network self-test, the events-per-thread tables,
 * the VEGAS grid refinement) run on real data.  A sanitizer report aborts the
 * program; otherwise it prints "sanitized abi ok".
 *
 * Test infrastructure: built and run by tests/test_sanitize.py only.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hydra_phsp.h"
#include "hydra_phsp_batch.h"
#include "hydra_phsp_model.h"
#include "hydra_phsp_probe.h"
#include "hydra_phsp_serve.h"
#include "hydra_phsp_unweight.h"
#include "hydra_phsp_vegas.h"

static int failures = 0;

static void expect(int cond, const char *what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s (last error: %s)\n", what, hydra_phsp_last_error());
        ++failures;
    }
}

#define FAKE(T, a) ((T *)(uintptr_t)(a))

static int gen(double M, const double *m, int n, uint64_t nev, uint64_t ld, uintptr_t out, uintptr_t w,
               const double *p4h, uintptr_t p4d, uint64_t ldp)
{
    return hydra_phsp_generate(M, m, n, p4h, FAKE(const double, p4d), ldp, nev, 1, 0, 0, FAKE(double, out), ld,
                               FAKE(double, w), NULL, NULL);
}

static void single_channel(void)
{
    const double two[2] = { 1.0, 1.0 }, heavy[2] = { 3.0, 2.5 }, neg[2] = { 1.0, -0.1 };
    double eleven[11];
    for (int i = 0; i < 11; ++i) eleven[i] = 0.1;
    const double p4_wrong_mass[4] = { 5.0, 1.0, 0.0, 0.0 }, p4_rest[4] = { 5.0, 0.0, 0.0, 0.0 };
    expect(gen(5.0, two, 1, 10, 10, 0x100, 0x100, NULL, 0, 0) == HYDRA_PHSP_EINVAL, "one daughter");
    expect(gen(50.0, eleven, 11, 10, 10, 0x100, 0x100, NULL, 0, 0) == HYDRA_PHSP_EINVAL, "eleven daughters");
    expect(gen(5.0, neg, 2, 10, 10, 0x100, 0x100, NULL, 0, 0) == HYDRA_PHSP_EINVAL, "negative mass");
    expect(gen(5.0, heavy, 2, 10, 10, 0x100, 0x100, NULL, 0, 0) == HYDRA_PHSP_EKINEMATICS, "below threshold");
    expect(gen(5.0, two, 2, 10, 5, 0x100, 0x100, NULL, 0, 0) == HYDRA_PHSP_EINVAL, "ld < nevents");
    expect(gen(5.0, two, 2, 10, 10, 0, 0x100, NULL, 0, 0) == HYDRA_PHSP_EINVAL, "null output");
    expect(gen(5.0, two, 2, 10, 10, 0x100, 0, NULL, 0, 0) == HYDRA_PHSP_EINVAL, "null weights");
    expect(gen(5.0, two, 2, 10, 10, 0x100, 0x100, p4_wrong_mass, 0, 0) == HYDRA_PHSP_EINVAL, "parent mass");
    expect(gen(5.0, two, 2, 10, 10, 0x100, 0x100, p4_rest, 0x100, 10) == HYDRA_PHSP_EINVAL, "two parent forms");
    expect(gen(5.0, two, 2, 10, 10, 0x100, 0x100, NULL, 0x100, 3) == HYDRA_PHSP_EINVAL, "short ld_parent");
    expect(gen(5.0, two, 2, 10, 10, 0x10c, 0x100, NULL, 0, 0) == HYDRA_PHSP_EINVAL, "misaligned output");
    expect(gen(5.0, two, 2, 10, 10, 0x100, 0x104, NULL, 0, 0) == HYDRA_PHSP_EINVAL, "misaligned weights");
    expect(gen(5.0, two, 2, ~0ull, ~0ull, 0x100, 0x100, NULL, 0, 0) == HYDRA_PHSP_EINVAL, "count beyond a launch");
    expect(hydra_phsp_generate_mixed(5.0, two, 2, NULL, NULL, 0, 10, 1, 0, 0, FAKE(float, 0x102), 10,
                                     FAKE(double, 0x100), NULL, NULL) == HYDRA_PHSP_EINVAL, "mixed misaligned");
    expect(hydra_phsp_generate_mixed(5.0, heavy, 2, NULL, NULL, 0, 10, 1, 0, 0, FAKE(float, 0x100), 10,
                                     FAKE(double, 0x100), NULL, NULL) == HYDRA_PHSP_EKINEMATICS, "mixed threshold");
    expect(hydra_phsp_generate_noalloc(5.0, two, 2, NULL, NULL, 0, 1ull << 40, 1, 0, 0, FAKE(double, 0x100),
                                       1ull << 40, FAKE(double, 0x100), NULL, NULL) == HYDRA_PHSP_EINVAL,
           "noalloc beyond its scratch");
    expect(hydra_phsp_generate_noalloc(5.0, neg, 2, NULL, NULL, 0, 10, 1, 0, 0, FAKE(double, 0x100), 10,
                                       FAKE(double, 0x100), NULL, NULL) == HYDRA_PHSP_EINVAL, "noalloc mass");
    double mean = 0.0, sigma = 0.0;
    expect(hydra_phsp_integrate(5.0, two, 2, 1, 1, 0, 0, &mean, &sigma, NULL) == HYDRA_PHSP_EINVAL,
           "integrate of one event");
    expect(hydra_phsp_integrate(5.0, two, 2, 10, 1, 0, 0, NULL, &sigma, NULL) == HYDRA_PHSP_EINVAL,
           "integrate without mean");
    expect(hydra_phsp_integrate_async(5.0, two, 2, 10, 1, 0, 0, NULL, NULL) == HYDRA_PHSP_EINVAL,
           "integrate_async without stats");
    expect(hydra_phsp_integrate_async(5.0, heavy, 2, 10, 1, 0, 0, FAKE(double, 0x100), NULL) ==
               HYDRA_PHSP_EKINEMATICS, "integrate_async threshold");
}

static void host_tables(void)
{
    for (int s = -7; s <= 1; ++s) expect(hydra_phsp_strerror(s) != NULL && strlen(hydra_phsp_strerror(s)) > 0,
                                          "strerror text");
    expect(hydra_phsp_strerror(-1000) != NULL, "strerror of an unknown code");
    expect(hydra_phsp_abi_version() == HYDRA_PHSP_ABI_VERSION, "abi version");
    expect(hydra_phsp_selftest_sortnet() == HYDRA_PHSP_OK, "sorting networks (0-1 principle)");
    for (int path = 0; path <= 2; ++path)
        for (int n = 2; n <= HYDRA_PHSP_NMAX; ++n)
            for (int flags = 0; flags <= 3; ++flags) {
                const int e = hydra_phsp_events_per_thread(path, n, flags);
                expect(e == 1 || e == 2 || e == 4, "events per thread");
            }
    expect(hydra_phsp_events_per_thread(3, 3, 0) == HYDRA_PHSP_EINVAL, "unknown path");
    expect(hydra_phsp_events_per_thread(1, 11, 0) == HYDRA_PHSP_EINVAL, "N = 11");
    expect(hydra_phsp_events_per_thread(1, 3, 4) == HYDRA_PHSP_EINVAL, "unknown flag");
    expect(hydra_phsp_set_events_per_thread(1, 3) == HYDRA_PHSP_EINVAL, "three events per thread");
    expect(hydra_phsp_set_events_per_thread(1, 2) == HYDRA_PHSP_OK, "set two events per thread");
    expect(hydra_phsp_events_per_thread(1, 3, 0) == 2, "override visible");
    expect(hydra_phsp_set_events_per_thread(1, 0) == HYDRA_PHSP_OK, "restore defaults");
    expect(hydra_phsp_set_unweight_chunks(17) == HYDRA_PHSP_EINVAL, "17 unweighting chunks");
    expect(hydra_phsp_set_unweight_chunks(-1) == HYDRA_PHSP_EINVAL, "negative unweighting chunks");
    expect(hydra_phsp_set_unweight_chunks(16) == HYDRA_PHSP_OK && hydra_phsp_set_unweight_chunks(0) == HYDRA_PHSP_OK,
           "unweighting chunks set and restored");
    {
        /* statistics of {1, 2} and {3, 4, 5}: union {1..5}, mean 3, M2 10 */
        double a[HYDRA_PHSP_STATS] = {2.0, 1.5, 0.5, 0.0}, b[HYDRA_PHSP_STATS] = {3.0, 4.0, 2.0, 0.0};
        double u[HYDRA_PHSP_STATS];
        expect(hydra_phsp_stats_merge(a, b, u) == HYDRA_PHSP_OK && u[0] == 5.0 && u[1] == 3.0 && u[2] == 10.0,
               "stats merge of {1,2} and {3,4,5}");
        expect(hydra_phsp_stats_merge(a, b, a) == HYDRA_PHSP_OK && a[1] == 3.0, "stats merge in place");
        double bad[HYDRA_PHSP_STATS] = {-1.0, 0.0, 0.0, 0.0};
        expect(hydra_phsp_stats_merge(bad, b, u) == HYDRA_PHSP_EINVAL, "stats merge of a negative n");
        expect(hydra_phsp_stats_merge(NULL, b, u) == HYDRA_PHSP_EINVAL, "stats merge of NULL");
    }
    expect(hydra_phsp_timing_enable(1) == HYDRA_PHSP_OK && hydra_phsp_timing_reset() == HYDRA_PHSP_OK,
           "timing switch");
    double ms = -1.0;
    uint64_t launches = 99;
    expect(hydra_phsp_timing_read(&ms, &launches) == HYDRA_PHSP_OK && launches == 0, "no timed launches");
    expect(hydra_phsp_timing_read(NULL, &launches) == HYDRA_PHSP_EINVAL, "timing_read without output");
    expect(hydra_phsp_timing_enable(0) == HYDRA_PHSP_OK, "timing off");
}

static void batched(void)
{
    hydra_phsp_channel ch[3];
    memset(ch, 0, sizeof(ch));
    for (int c = 0; c < 3; ++c) {
        ch[c].parent_mass = 5.0;
        ch[c].n_daughters = 2;
        ch[c].masses[0] = 1.0;
        ch[c].masses[1] = 1.0;
        ch[c].nevents = 100;
        ch[c].p4_out_dev = FAKE(double, 0x1000);
        ch[c].ld = 128;
        ch[c].weights_dev = FAKE(double, 0x2000);
        ch[c].stats_dev = FAKE(double, 0x3000);
    }
    ch[1].masses[1] = 4.5; /* above threshold: channel 1 is the bad one */
    int bad = -1;
    expect(hydra_phsp_batch_run(ch, 3, NULL, NULL, &bad) == HYDRA_PHSP_EKINEMATICS && bad == 1,
           "batch names its bad channel");
    ch[1].masses[1] = 1.0;
    ch[2].ld = 50;
    expect(hydra_phsp_batch_run(ch, 3, NULL, NULL, &bad) == HYDRA_PHSP_EINVAL && bad == 2, "batch ld");
    ch[2].ld = 128;
    expect(hydra_phsp_batch_run(ch, 0, NULL, NULL, &bad) == HYDRA_PHSP_EINVAL, "empty batch");
    expect(hydra_phsp_batch_run(NULL, 3, NULL, NULL, &bad) == HYDRA_PHSP_EINVAL, "null channels");
    hydra_phsp_tuning t = { 3, 0, 0, 0 };
    expect(hydra_phsp_batch_run(ch, 3, &t, NULL, &bad) == HYDRA_PHSP_EINVAL, "tuning ept 3");
    t.ept = 0;
    t.schedule = 9;
    expect(hydra_phsp_batch_run(ch, 3, &t, NULL, &bad) == HYDRA_PHSP_EINVAL, "unknown schedule");
    t.schedule = 0;
    t.streams = HYDRA_PHSP_MAX_CLASS_STREAMS + 1;
    expect(hydra_phsp_batch_run(ch, 3, &t, NULL, &bad) == HYDRA_PHSP_EINVAL, "too many streams");
    hydra_phsp_plan *plan = NULL;
    ch[0].n_daughters = 12;
    expect(hydra_phsp_plan_create(ch, 3, NULL, &plan) == HYDRA_PHSP_EINVAL && plan == NULL, "plan of a bad batch");
    expect(hydra_phsp_plan_create(ch, 3, NULL, NULL) == HYDRA_PHSP_EINVAL, "plan without output");
    expect(hydra_phsp_plan_launch(NULL, NULL) == HYDRA_PHSP_EINVAL, "launch of no plan");
    uint64_t a, b;
    expect(hydra_phsp_plan_info(NULL, &a, &b) == HYDRA_PHSP_EINVAL, "info of no plan");
    hydra_phsp_tuning best;
    double best_ms;
    expect(hydra_phsp_autotune(ch, 3, NULL, &best, &best_ms) == HYDRA_PHSP_EINVAL, "autotune of a bad batch");
    expect(hydra_phsp_autotune(ch, 3, NULL, NULL, &best_ms) == HYDRA_PHSP_EINVAL, "autotune without output");
}

static void next_rows(void)
{
    const double m3[3] = { 3.097, 0.4937, 0.13957 };
    expect(hydra_phsp_generate_unweighted(5.279, m3, 3, NULL, 100, 42, 0, 0, -1.0, FAKE(double, 0x100), 128, NULL,
                                          FAKE(uint64_t, 0x200), FAKE(double, 0x300), NULL) == HYDRA_PHSP_EINVAL,
           "negative bound");
    expect(hydra_phsp_generate_unweighted(5.279, m3, 3, NULL, 100, 42, 0, 0, 0.0, FAKE(double, 0x100), 128, NULL,
                                          NULL, FAKE(double, 0x300), NULL) == HYDRA_PHSP_EINVAL, "no counts");
    hydra_phsp_breit_wigner bw[HYDRA_PHSP_MAX_BW + 1];
    for (int k = 0; k <= HYDRA_PHSP_MAX_BW; ++k) {
        bw[k].i = 1;
        bw[k].j = 2;
        bw[k].mass = 0.8955;
        bw[k].width = 0.0473;
    }
    expect(hydra_phsp_integrate_model(5.279, m3, 3, bw, HYDRA_PHSP_MAX_BW + 1, 100, 42, 0, 0, NULL,
                                      FAKE(double, 0x100), NULL) == HYDRA_PHSP_EINVAL, "too many factors");
    bw[0].j = 3;
    expect(hydra_phsp_integrate_model(5.279, m3, 3, bw, 1, 100, 42, 0, 0, NULL, FAKE(double, 0x100), NULL) ==
               HYDRA_PHSP_EINVAL, "daughter index out of range");
    bw[0].j = 2;
    bw[0].width = 0.0;
    expect(hydra_phsp_integrate_model(5.279, m3, 3, bw, 1, 100, 42, 0, 0, NULL, FAKE(double, 0x100), NULL) ==
               HYDRA_PHSP_EINVAL, "zero width");
    expect(hydra_phsp_generate_unweighted_model(5.279, m3, 3, bw, 1, 100, 42, 0, 0, 0.0, FAKE(double, 0x100), 128,
                                                NULL, FAKE(uint64_t, 0x200), NULL, NULL) == HYDRA_PHSP_EINVAL,
           "unweighted model with a zero width");
    bw[0].width = 0.0473;
    expect(hydra_phsp_generate_unweighted_model(5.279, m3, 3, bw, HYDRA_PHSP_MAX_BW + 1, 100, 42, 0, 0, 0.0,
                                                FAKE(double, 0x100), 128, NULL, FAKE(uint64_t, 0x200), NULL,
                                                NULL) == HYDRA_PHSP_EINVAL, "unweighted model, too many factors");
    expect(hydra_phsp_generate_unweighted_model(5.279, m3, 3, bw, 1, 100, 42, 0, 0, 0.0, FAKE(double, 0x100), 128,
                                                NULL, NULL, NULL, NULL) == HYDRA_PHSP_EINVAL,
           "unweighted model without counts");

    /* VEGAS: the refinement is host code; run it on real grids and histograms */
    enum { D = 3, K = 11 };
    double grid[D * (K + 1)], hist[D * K];
    for (int d = 0; d < D; ++d)
        for (int k = 0; k <= K; ++k) grid[d * (K + 1) + k] = (double)k / K;
    for (int round = 0; round < 4; ++round) {
        for (int i = 0; i < D * K; ++i) hist[i] = (round == 1) ? 0.0 : (double)((i * 7 + round) % 5);
        if (round == 2) hist[4] = 1e300;
        expect(hydra_phsp_vegas_refine(D, K, grid, hist, 1.5) == HYDRA_PHSP_OK, "refinement");
        for (int d = 0; d < D; ++d) {
            expect(grid[d * (K + 1)] == 0.0 && grid[d * (K + 1) + K] == 1.0, "grid ends");
            for (int k = 0; k < K; ++k) expect(grid[d * (K + 1) + k] < grid[d * (K + 1) + k + 1], "monotone grid");
        }
    }
    expect(hydra_phsp_vegas_refine(D, 0, grid, hist, 1.5) == HYDRA_PHSP_EINVAL, "zero bins");
    expect(hydra_phsp_vegas_refine(HYDRA_PHSP_VEGAS_DMAX + 1, K, grid, hist, 1.5) == HYDRA_PHSP_EINVAL,
           "too many dimensions");
    expect(hydra_phsp_vegas_refine(D, K, NULL, hist, 1.5) == HYDRA_PHSP_EINVAL, "no grid");
    hydra_phsp_gauss_box f;
    memset(&f, 0, sizeof(f));
    f.dim = D;
    for (int d = 0; d < D; ++d) {
        f.lo[d] = 0.0;
        f.hi[d] = 1.0;
        f.mean[d] = 0.5;
        f.sigma[d] = 0.1;
    }
    f.sigma[1] = 0.0;
    expect(hydra_phsp_vegas_iteration(&f, K, FAKE(const double, 0x100), 1000, 42, 0, FAKE(double, 0x200), NULL,
                                      NULL, NULL) == HYDRA_PHSP_EINVAL, "zero sigma");
    f.sigma[1] = 0.1;
    expect(hydra_phsp_vegas_iteration(&f, K, FAKE(const double, 0x100), 1, 42, 0, FAKE(double, 0x200), NULL,
                                      NULL, NULL) == HYDRA_PHSP_EINVAL, "one call");
    double res, err, chi;
    expect(hydra_phsp_vegas(&f, K, 1000, 0, 0, 1.5, 42, grid, &res, &err, &chi, NULL) == HYDRA_PHSP_EINVAL,
           "no estimating iteration");
    expect(hydra_phsp_probe_write(FAKE(double, 0x100), 10, 0, FAKE(double, 0x200), 10, 1, NULL) ==
               HYDRA_PHSP_EINVAL, "probe without columns");
    expect(hydra_phsp_probe_philox(10, 0, 42, 0, FAKE(uint32_t, 0x100), NULL) == HYDRA_PHSP_EINVAL,
           "probe without calls");
}

static void serving(void)
{
    hydra_phsp_server *s = NULL;
    expect(hydra_phsp_server_create(0, 0, 0, &s) == HYDRA_PHSP_EINVAL && s == NULL, "server without budget");
    expect(hydra_phsp_server_create(1 << 20, 0, 0, NULL) == HYDRA_PHSP_EINVAL, "server without output");
    hydra_phsp_request r;
    memset(&r, 0, sizeof(r));
    uint64_t id;
    expect(hydra_phsp_server_submit(NULL, &r, &id) == HYDRA_PHSP_EINVAL, "submit to no server");
    expect(hydra_phsp_server_step(NULL) == HYDRA_PHSP_EINVAL, "step of no server");
    hydra_phsp_result res;
    expect(hydra_phsp_server_poll(NULL, 1, &res) == HYDRA_PHSP_EINVAL, "poll of no server");
    expect(hydra_phsp_server_release(NULL, 1) == HYDRA_PHSP_EINVAL, "release on no server");
    expect(hydra_phsp_server_drain(NULL) == HYDRA_PHSP_EINVAL, "drain of no server");
    hydra_phsp_server_counters c;
    expect(hydra_phsp_server_counters_get(NULL, &c) == HYDRA_PHSP_EINVAL, "counters of no server");
}

/* User intensities: compilation (hiprtc, host only), the compiler's log for a
 * bad source, and validation of every evaluation argument before the code
 * object is loaded. */
static void user_models(void)
{
    static const char good[] =
        "__device__ double hydra_phsp_user_intensity(const double* e, const double* px, const double* py,\n"
        "    const double* pz, const double* par) { return par[0] * e[0] + pz[1] * pz[1]; }\n";
    hydra_phsp_user_model *um = NULL;
    expect(hydra_phsp_user_model_create(good, 3, &um) == HYDRA_PHSP_OK && um != NULL, "user model compiles");
    expect(hydra_phsp_user_model_daughters(um) == 3, "user model daughters");
    const double m3[3] = { 3.097, 0.4937, 0.13957 };
    double par[HYDRA_PHSP_USER_PARAMS + 1];
    for (int k = 0; k <= HYDRA_PHSP_USER_PARAMS; ++k) par[k] = 0.5;
    expect(hydra_phsp_integrate_user_model(um, 5.279, m3, par, HYDRA_PHSP_USER_PARAMS + 1, 100, 42, 0, 0, NULL,
                                           FAKE(double, 0x100), NULL) == HYDRA_PHSP_EINVAL, "too many parameters");
    expect(hydra_phsp_integrate_user_model(um, 5.279, m3, NULL, 2, 100, 42, 0, 0, NULL, FAKE(double, 0x100),
                                           NULL) == HYDRA_PHSP_EINVAL, "no parameters");
    expect(hydra_phsp_integrate_user_model(um, 5.279, m3, par, 2, 100, 42, 0, 0, NULL, NULL, NULL) ==
               HYDRA_PHSP_EINVAL, "no stats");
    expect(hydra_phsp_integrate_user_model(um, 3.5, m3, par, 2, 100, 42, 0, 0, NULL, FAKE(double, 0x100), NULL) ==
               HYDRA_PHSP_EKINEMATICS, "user model kinematics");
    expect(hydra_phsp_integrate_user_model(NULL, 5.279, m3, par, 2, 100, 42, 0, 0, NULL, FAKE(double, 0x100),
                                           NULL) == HYDRA_PHSP_EINVAL, "no user model");
    expect(hydra_phsp_generate_unweighted_user_model(um, 5.279, m3, par, HYDRA_PHSP_USER_PARAMS + 1, 100, 42, 0, 0,
                                                     0.0, FAKE(double, 0x100), 128, NULL, FAKE(uint64_t, 0x200),
                                                     NULL, NULL) == HYDRA_PHSP_EINVAL,
           "unweighted user model, too many parameters");
    expect(hydra_phsp_generate_unweighted_user_model(um, 5.279, m3, par, 2, 100, 42, 0, 0, -1.0,
                                                     FAKE(double, 0x100), 128, NULL, FAKE(uint64_t, 0x200), NULL,
                                                     NULL) == HYDRA_PHSP_EINVAL, "unweighted user model bound");
    expect(hydra_phsp_generate_unweighted_user_model(NULL, 5.279, m3, par, 2, 100, 42, 0, 0, 0.0,
                                                     FAKE(double, 0x100), 128, NULL, FAKE(uint64_t, 0x200), NULL,
                                                     NULL) == HYDRA_PHSP_EINVAL, "unweighted without user model");
    expect(hydra_phsp_user_model_destroy(um) == HYDRA_PHSP_OK, "user model destroy");
    hydra_phsp_user_model *bad = NULL;
    expect(hydra_phsp_user_model_create("not a function at all", 3, &bad) == HYDRA_PHSP_EINVAL && bad == NULL,
           "bad source");
    expect(strstr(hydra_phsp_last_error(), "does not compile") != NULL, "compiler log");
    expect(hydra_phsp_user_model_create(good, 11, &bad) == HYDRA_PHSP_EINVAL, "user model daughters range");
    expect(hydra_phsp_user_model_destroy(NULL) == HYDRA_PHSP_EINVAL, "destroy of no model");

    static const char integrand[] =
        "__device__ double hydra_phsp_user_integrand(const double* x, const double* par)\n"
        "{ return x[0] * x[HYDRA_PHSP_DIM - 1] + par[0]; }\n";
    hydra_phsp_user_integrand *ui = NULL;
    expect(hydra_phsp_user_integrand_create(integrand, 3, &ui) == HYDRA_PHSP_OK && ui != NULL,
           "user integrand compiles");
    const double lo[3] = { 0.0, 0.0, -1.0 }, hi[3] = { 1.0, 2.0, 1.0 }, bad_hi[3] = { 1.0, 0.0, 1.0 };
    double r = 0.0, e = 0.0, c = 0.0;
    expect(hydra_phsp_vegas_user_iteration(ui, lo, bad_hi, par, 1, 10, FAKE(double, 0x100), 100, 1, 0,
                                           FAKE(double, 0x200), NULL, NULL, NULL) == HYDRA_PHSP_EINVAL, "bad box");
    expect(hydra_phsp_vegas_user_iteration(ui, lo, hi, par, HYDRA_PHSP_USER_PARAMS + 1, 10, FAKE(double, 0x100),
                                           100, 1, 0, FAKE(double, 0x200), NULL, NULL, NULL) == HYDRA_PHSP_EINVAL,
           "too many integrand parameters");
    expect(hydra_phsp_vegas_user_iteration(ui, lo, hi, par, 1, 10, FAKE(double, 0x100), 1, 1, 0,
                                           FAKE(double, 0x200), NULL, NULL, NULL) == HYDRA_PHSP_EINVAL, "one call");
    expect(hydra_phsp_vegas_user(ui, lo, hi, par, 1, 10, 100, 0, 0, 1.5, 1, NULL, &r, &e, &c, NULL) ==
               HYDRA_PHSP_EINVAL, "no estimating iteration");
    expect(hydra_phsp_vegas_user(NULL, lo, hi, par, 1, 10, 100, 0, 1, 1.5, 1, NULL, &r, &e, &c, NULL) ==
               HYDRA_PHSP_EINVAL, "no integrand");
    expect(hydra_phsp_user_integrand_destroy(ui) == HYDRA_PHSP_OK, "user integrand destroy");
    expect(hydra_phsp_user_integrand_create("double x(", 3, &ui) == HYDRA_PHSP_EINVAL, "bad integrand source");
    expect(hydra_phsp_user_integrand_destroy(NULL) == HYDRA_PHSP_EINVAL, "destroy of no integrand");
}

int main(void)
{
    host_tables();
    single_channel();
    batched();
    next_rows();
    serving();
    user_models();
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("sanitized abi ok\n");
    return 0;
}

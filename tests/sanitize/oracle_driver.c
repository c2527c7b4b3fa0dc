/*
 * oracle_driver.c -- exercises every entry point of the CPU oracle
 * (oracle/phsp_oracle.c) on small valid and invalid inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer.  A sanitizer report aborts
 * the program (-fno-sanitize-recover=all); otherwise it checks a few results
 * that hold for any correct run and prints "sanitized oracle ok".
 *
 * Test infrastructure: built and run by tests/test_sanitize.py only.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int oracle_uniforms_per_event(int n);
void oracle_event_uniforms(uint64_t seed, uint32_t stream_id, uint64_t g, int n, double *u);
double oracle_weight_constant(double parent_mass, const double *masses, int n);
int oracle_generate(double parent_mass, const double *masses, int n, const double *parent_p4,
                    const double *parent_soa, uint64_t ld_parent, uint64_t nevents, uint64_t seed,
                    uint32_t stream_id, uint64_t event_offset, double *out, uint64_t ld, double *weights);
int oracle_integrate(double parent_mass, const double *masses, int n, uint64_t nevents, uint64_t seed,
                     uint32_t stream_id, uint64_t event_offset, double *mean, double *sigma);
int oracle_calls_per_event(int n);
double oracle_accept_uniform(uint64_t seed, uint32_t stream_id, uint64_t g, int n);
int oracle_unweight(double parent_mass, const double *masses, int n, const double *parent_p4,
                    uint64_t ntrials, uint64_t seed, uint32_t stream_id, uint64_t event_offset,
                    double w_max, double *out, uint64_t ld, uint64_t *index, uint64_t counts[2],
                    double *w_max_used);
int oracle_model_integrate(double parent_mass, const double *masses, int n, int n_bw, const int *pi,
                           const int *pj, const double *mass, const double *width, uint64_t nevents,
                           uint64_t seed, uint32_t stream_id, uint64_t event_offset, double *values,
                           double *mean, double *sigma);
int oracle_vegas_iteration(int dim, int bins, const double *lo, const double *hi, const double *mu,
                           const double *sig, const double *grid, uint64_t calls, uint64_t seed,
                           uint32_t iteration, double *mean, double *sigma, double *hist, double *values);
int oracle_vegas_refine(int dim, int bins, double *grid, const double *hist, double alpha);

static int failures = 0;

static void expect(int cond, const char *what)
{
    if (!cond) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

/* Every buffer is allocated at exactly the size the call needs, so any
 * out-of-bounds access by the oracle lands in a redzone. */
static void generate_cases(void)
{
    const double m3[3] = { 3.097, 0.4937, 0.13957 };
    const uint64_t nev = 257, ld = 259;
    for (int n = 2; n <= 10; ++n) {
        double masses[10];
        for (int i = 0; i < n; ++i) masses[i] = (n == 3) ? m3[i] : 0.13957 * (i % 2);
        const double M = (n == 3) ? 5.279 : 10.0;
        double *out = malloc(sizeof(double) * 4 * (size_t)n * ld);
        double *w = malloc(sizeof(double) * nev);
        double *par = malloc(sizeof(double) * 4 * ld);
        for (uint64_t e = 0; e < ld; ++e) {
            const double pz = 20.0 * (double)e / (double)ld;
            par[0 * ld + e] = sqrt(M * M + pz * pz);
            par[1 * ld + e] = 0.0;
            par[2 * ld + e] = 0.0;
            par[3 * ld + e] = pz;
        }
        const double p4[4] = { sqrt(M * M + 4.0), 1.0, -1.0, 1.4142135623730951 };
        expect(oracle_generate(M, masses, n, NULL, NULL, 0, nev, 42, 0, 0, out, ld, w) == 0, "generate at rest");
        for (uint64_t e = 0; e < nev; ++e) expect(w[e] > 0.0 && isfinite(w[e]), "positive weight");
        expect(oracle_generate(M, masses, n, p4, NULL, 0, nev, 42, 1, (1ull << 32) - 100, out, ld, w) == 0,
               "generate broadcast parent");
        expect(oracle_generate(M, masses, n, NULL, par, ld, nev, 42, 2, 0, out, ld, w) == 0,
               "generate per-event parents");
        expect(oracle_generate(M, masses, n, NULL, NULL, 0, nev, 7, 0, 0, NULL, 0, w) == 0, "weights only");
        double mean = 0.0, sigma = 0.0;
        expect(oracle_integrate(M, masses, n, nev, 42, 0, 5, &mean, &sigma) == 0 && mean > 0.0, "integrate");
        expect(oracle_weight_constant(M, masses, n) > 0.0, "weight constant");
        double *u = malloc(sizeof(double) * (size_t)oracle_uniforms_per_event(n));
        oracle_event_uniforms(42, 0, 12345, n, u);
        for (int k = 0; k < oracle_uniforms_per_event(n); ++k) expect(u[k] > 0.0 && u[k] < 1.0, "open uniform");
        free(u);
        free(out);
        free(w);
        free(par);
    }
    /* invalid arguments: rejected before any access */
    const double bad[3] = { 3.097, -0.5, 0.13957 };
    double w1[4];
    double out1[48];
    expect(oracle_generate(5.279, bad, 3, NULL, NULL, 0, 4, 42, 0, 0, out1, 4, w1) != 0, "negative mass");
    expect(oracle_generate(1.0, m3, 3, NULL, NULL, 0, 4, 42, 0, 0, out1, 4, w1) != 0, "below threshold");
    expect(oracle_generate(5.279, m3, 11, NULL, NULL, 0, 4, 42, 0, 0, out1, 4, w1) != 0, "too many daughters");
    expect(oracle_generate(5.279, m3, 3, NULL, NULL, 0, 4, 42, 0, 0, out1, 3, w1) != 0, "ld < nevents");
    double mean, sigma;
    expect(oracle_integrate(5.279, m3, 3, 1, 42, 0, 0, &mean, &sigma) != 0, "integrate of one event");
}

static void unweight_cases(void)
{
    const double m3[3] = { 3.097, 0.4937, 0.13957 };
    const uint64_t ntr = 1000;
    for (int cap = 0; cap <= 1; ++cap) {
        const uint64_t ld = cap ? 37 : ntr;
        double *out = malloc(sizeof(double) * 12 * ld);
        uint64_t *idx = malloc(sizeof(uint64_t) * ld);
        uint64_t counts[2];
        double wmax = 0.0;
        expect(oracle_unweight(5.279, m3, 3, NULL, ntr, 42, 0, 0, 0.0, out, ld, idx, counts, &wmax) == 0,
               "unweight with sample maximum");
        expect(counts[0] >= 1 && counts[0] <= ntr && wmax > 0.0, "kept count");
        expect(oracle_unweight(5.279, m3, 3, NULL, ntr, 42, 0, 0, 0.5 * wmax, out, ld, idx, counts, &wmax) == 0,
               "unweight with a low bound");
        expect(counts[1] > 0, "over-bound trials counted");
        free(out);
        free(idx);
    }
    expect(oracle_calls_per_event(3) == 3 && oracle_calls_per_event(10) == 13, "calls per event");
    const double v = oracle_accept_uniform(42, 0, 99, 3);
    expect(v > 0.0 && v < 1.0, "acceptance uniform");
}

static void model_cases(void)
{
    const double m3[3] = { 3.097, 0.4937, 0.13957 };
    const uint64_t nev = 300;
    const int pi[2] = { 1, 0 }, pj[2] = { 2, 1 };
    const double bm[2] = { 0.8955, 3.686 }, bw[2] = { 0.0473, 0.3 };
    double *vals = malloc(sizeof(double) * nev);
    double mean, sigma;
    for (int k = 0; k <= 2; ++k)
        expect(oracle_model_integrate(5.279, m3, 3, k, pi, pj, bm, bw, nev, 42, 0, 0, vals, &mean, &sigma) == 0,
               "model integral");
    const int bad_i[1] = { 3 }, bad_j[1] = { 0 };
    expect(oracle_model_integrate(5.279, m3, 3, 1, bad_i, bad_j, bm, bw, nev, 42, 0, 0, vals, &mean, &sigma) != 0,
           "daughter index out of range");
    free(vals);
}

static void vegas_cases(void)
{
    enum { D = 4, K = 7 };
    const uint64_t calls = 500;
    double lo[D], hi[D], mu[D], sg[D];
    for (int d = 0; d < D; ++d) {
        lo[d] = 0.0;
        hi[d] = 1.0;
        mu[d] = 0.5;
        sg[d] = 0.1;
    }
    double *grid = malloc(sizeof(double) * D * (K + 1));
    for (int d = 0; d < D; ++d)
        for (int k = 0; k <= K; ++k) grid[d * (K + 1) + k] = (double)k / K;
    double *hist = malloc(sizeof(double) * D * K);
    double *vals = malloc(sizeof(double) * calls);
    double mean, sigma;
    for (int it = 0; it < 3; ++it) {
        expect(oracle_vegas_iteration(D, K, lo, hi, mu, sg, grid, calls, 42, (uint32_t)it, &mean, &sigma, hist,
                                      vals) == 0, "vegas iteration");
        expect(oracle_vegas_refine(D, K, grid, hist, 1.5) == 0, "vegas refinement");
        for (int d = 0; d < D; ++d)
            for (int k = 0; k < K; ++k)
                expect(grid[d * (K + 1) + k] < grid[d * (K + 1) + k + 1], "monotone grid");
    }
    /* a histogram that is empty except one bin, and an all-zero one */
    for (int i = 0; i < D * K; ++i) hist[i] = 0.0;
    expect(oracle_vegas_refine(D, K, grid, hist, 1.5) == 0, "refinement of an empty histogram");
    hist[3] = 1.0;
    expect(oracle_vegas_refine(D, K, grid, hist, 1.5) == 0, "refinement of a single spike");
    expect(oracle_vegas_iteration(D, 0, lo, hi, mu, sg, grid, calls, 42, 0, &mean, &sigma, hist, vals) != 0,
           "zero bins");
    free(grid);
    free(hist);
    free(vals);
}

int main(void)
{
    const uint32_t ctr[4] = { 1, 2, 3, 4 }, key[2] = { 5, 6 };
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    generate_cases();
    unweight_cases();
    model_cases();
    vegas_cases();
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("sanitized oracle ok\n");
    return 0;
}

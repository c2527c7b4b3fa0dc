/*
 * phsp_oracle.c -- plain, slow, single-threaded FP64 CPU oracle for N-body
 * phase-space Monte Carlo generation and integration (Raubold-Lynch method,
 * arXiv:1711.05683 sec. 4.2 "Phase-Space Monte Carlo").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; the two sides meet
 * only through seeded inputs and the counter-based generator each implements
 * from its published definition.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math), so that every
 * operation below is one IEEE-754 round-to-nearest double operation, evaluated
 * in the order written.
 *
 * What the paper fixes and what is a reading of it
 * ------------------------------------------------
 * Sec. 4.2 states the problem (a particle of given four-momentum decaying to an
 * n-body final state with no intermediate resonances), names the method
 * (Raubold-Lynch, after F. James, CERN 68-15), says any number of daughters is
 * supported and that weighted samples are produced.  Listing "lst:phsp" shows
 * the interface: parent mass and daughter masses at construction, a parent
 * four-vector Vector4R(mass,0,0,0) (energy first) at generation time, and a
 * caller-allocated event container.  Everything else -- random-number
 * generator, uniform conversion, recursion order, angle convention, weight
 * normalisation -- is silent in the paper; this file makes the following
 * choices, each restated where it is used:
 *
 *  - phase-space measure: prod_i d^3p_i/(2E_i) delta^4(P - sum p_i), no 2*pi
 *    factors, so the two-body volume is pi*p/M and the mean weight is the
 *    N-body volume R_N (recursive factorisation of Lorentz-invariant phase
 *    space, the basis of the Raubold-Lynch method);
 *  - random words: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 *    Random Numbers: As Easy as 1, 2, 3", SC'11), key = 64-bit seed,
 *    counter = (low 32 bits of g, high 32 bits of g, call index j, stream id),
 *    g = event_offset + local event index;
 *  - uniform k from words 2k, 2k+1: 52 bits x, u = (2x+1) 2^-53 in (0,1);
 *  - the first N-2 uniforms are the mass uniforms; then (theta, phi) pairs for
 *    levels 0..N-2;
 *  - daughter 0 is innermost; the levels are built from the top down: each
 *    subsystem {0..i+1} splits, in its own rest frame (reached from the
 *    parent's rest frame by one pure boost), into daughter i+1 and {0..i},
 *    and both are boosted back into the parent's rest frame, so every
 *    daughter takes one boost (the chain runs through the subsystems'
 *    four-momenta).  For three daughters this is the same as boosting the
 *    inner pair up level by level; for more it is an equally valid
 *    parametrisation of the same phase space (every direction is isotropic in
 *    its subsystem's rest frame whatever that frame's orientation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_NMAX 10
/* pi to double precision (the double nearest pi) */
static const double ORACLE_PI = 3.141592653589793;

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (SC'11 paper, section 3.2 "Philox"): 10 rounds of a       */
/* two-multiplier S-box/P-box on a 4x32-bit counter, 2x32-bit key bumped   */
/* by the Weyl constants between rounds.                                   */
/* ---------------------------------------------------------------------- */
static const uint32_t PHILOX_M0 = 0xD2511F53u; /* multiplier applied to word 0 */
static const uint32_t PHILOX_M1 = 0xCD9E8D57u; /* multiplier applied to word 2 */
static const uint32_t PHILOX_W0 = 0x9E3779B9u; /* key bump, word 0 (golden ratio) */
static const uint32_t PHILOX_W1 = 0xBB67AE85u; /* key bump, word 1 (sqrt(3)-1) */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t prod0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t prod1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Number of random uniforms one event consumes: N-2 mass uniforms plus a
 * (theta, phi) pair for each of the N-1 two-body levels. */
int oracle_uniforms_per_event(int n)
{
    return 3 * n - 4;
}

/* Uniforms of global event g: u[k] for k = 0 .. 3N-5.  Each uniform takes two
 * consecutive 32-bit words (low word first) of the event's Philox stream; the
 * stream is call j = 0, 1, ... of the counter (g_lo, g_hi, j, stream_id). */
void oracle_event_uniforms(uint64_t seed, uint32_t stream_id, uint64_t g, int n, double *u)
{
    const int nu = oracle_uniforms_per_event(n);
    const int nwords = 2 * nu;
    uint32_t words[4 * ((2 * (3 * ORACLE_NMAX - 4) + 3) / 4)];
    const uint32_t key[2] = { (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32) };
    for (int j = 0; 4 * j < nwords; ++j) {
        const uint32_t ctr[4] = { (uint32_t)(g & 0xFFFFFFFFu), (uint32_t)(g >> 32),
                                  (uint32_t)j, stream_id };
        oracle_philox4x32_10(ctr, key, &words[4 * j]);
    }
    for (int k = 0; k < nu; ++k) {
        uint64_t bits = ((uint64_t)words[2 * k + 1] << 32) | (uint64_t)words[2 * k];
        uint64_t x = bits >> 12;                     /* 52 bits */
        u[k] = (double)(2 * x + 1) * 0x1p-53;        /* exact, in [2^-53, 1-2^-53] */
    }
}

/* Normalisation of the weight.  Unrolling the recursion
 *   R_N(M) = int d(sigma^2) R_2(M; sigma, m_{N-1}) R_{N-1}(sigma; m_0..m_{N-2}),
 *   R_2(a; b, c) = pi p(a; b, c) / a,
 * and substituting sigma_i = S_i + T R_i (sorted R on the unit simplex of
 * volume 1/(N-2)!) leaves
 *   R_N = pi^{N-1} (2T)^{N-2} / (M (N-2)!) * E[ prod_i p_i ].
 * The factors are multiplied in the order written in this comment. */
double oracle_weight_constant(double parent_mass, const double *masses, int n)
{
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += masses[i];
    const double t = parent_mass - s;
    double c = 1.0 / parent_mass;
    for (int i = 0; i < n - 1; ++i) c = c * ORACLE_PI;
    for (int i = 0; i < n - 2; ++i) c = c * (2.0 * t);
    double fact = 1.0;
    for (int i = 2; i <= n - 2; ++i) fact = fact * (double)i;
    return c / fact;
}

/* Ascending sort of a handful of doubles (insertion sort: obviously correct). */
static void sort_ascending(double *a, int n)
{
    for (int i = 1; i < n; ++i) {
        double v = a[i];
        int j = i - 1;
        while (j >= 0 && a[j] > v) {
            a[j + 1] = a[j];
            --j;
        }
        a[j + 1] = v;
    }
}

/* Pure Lorentz boost of the four-vector v = (E, px, py, pz) by rapidity vector
 * eta = gamma*beta: E' = gamma E + eta.p,  p' = p + (eta.p/(gamma+1) + E) eta. */
static void boost(double v[4], const double eta[3], double gamma)
{
    const double e = v[0];
    const double ep = eta[0] * v[1] + eta[1] * v[2] + eta[2] * v[3];
    const double f = ep / (gamma + 1.0) + e;
    v[0] = gamma * e + ep;
    v[1] = v[1] + f * eta[0];
    v[2] = v[2] + f * eta[1];
    v[3] = v[3] + f * eta[2];
}

/* Isotropic unit vector from two uniforms: cos(theta) = 2u - 1,
 * sin(theta) = 2 sqrt(u (1-u)), phi = 2 pi v. */
static void direction(double u, double v, double nhat[3])
{
    const double ct = 2.0 * u - 1.0;
    const double st = 2.0 * sqrt(u * (1.0 - u));
    const double phi = 6.283185307179586 * v;
    nhat[0] = st * cos(phi);
    nhat[1] = st * sin(phi);
    nhat[2] = ct;
}

/* One event.  p4[d][mu] receives daughter d's (E, px, py, pz) in the frame of
 * the parent given by (parent4 == NULL: at rest; else the parent's four-vector,
 * boosted with eta = P/M, gamma = E_P/M); the return value is the weight. */
static double one_event(double parent_mass, const double *masses, int n,
                        const double *parent4, const double *u, double p4[][4])
{
    double prefix[ORACLE_NMAX];                  /* S_i = m_0 + ... + m_i */
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        s += masses[i];
        prefix[i] = s;
    }
    const double t = parent_mass - s;            /* kinetic energy released */

    /* Sorted mass uniforms R_0 = 0 < R_1 <= ... <= R_{N-2} < R_{N-1} = 1. */
    double r[ORACLE_NMAX];
    r[0] = 0.0;
    for (int i = 0; i < n - 2; ++i) r[i + 1] = u[i];
    sort_ascending(&r[1], n - 2);
    r[n - 1] = 1.0;

    /* Invariant masses of the subsystems {0..i}. */
    double sigma[ORACLE_NMAX];
    sigma[0] = masses[0];
    for (int i = 1; i <= n - 2; ++i) sigma[i] = prefix[i] + t * r[i];
    sigma[n - 1] = parent_mass;

    /* Two-body breakup momentum of sigma_{i+1} -> sigma_i + m_{i+1}, with the
     * released energy g_i = sigma_{i+1} - sigma_i - m_{i+1} = T (R_{i+1} - R_i). */
    double p[ORACLE_NMAX];
    for (int i = 0; i <= n - 2; ++i) {
        const double gi = t * (r[i + 1] - r[i]);
        const double b = sigma[i], c = masses[i + 1];
        const double q = gi * (2.0 * b + 2.0 * c + gi) * (gi + 2.0 * c) * (2.0 * b + gi);
        p[i] = sqrt(q) / (2.0 * sigma[i + 1]);
    }

    double w = oracle_weight_constant(parent_mass, masses, n);
    for (int i = 0; i <= n - 2; ++i) w = w * p[i];

    /* Levels from the top down.  At level i the subsystem {0..i+1} (mass
     * sigma_{i+1}, four-momentum sub in the parent's rest frame; the parent
     * itself at the top) splits into daughter i+1 and the subsystem {0..i}
     * (daughter 0 when i = 0), back to back along nhat_i in the rest frame of
     * {0..i+1} that a pure boost reaches from the parent's rest frame.  Both
     * are boosted into the parent's rest frame with eta = sub/sigma_{i+1},
     * gamma = E_sub/sigma_{i+1} (nothing to do at the top); daughter i+1 is
     * then final and the subsystem goes down one level. */
    double sub[4] = { parent_mass, 0.0, 0.0, 0.0 };
    for (int i = n - 2; i >= 0; --i) {
        double nhat[3];
        direction(u[n - 2 + 2 * i], u[n - 1 + 2 * i], nhat);
        double dau[4], rest[4];
        dau[0] = sqrt(p[i] * p[i] + masses[i + 1] * masses[i + 1]);
        rest[0] = sqrt(p[i] * p[i] + sigma[i] * sigma[i]);
        for (int k = 0; k < 3; ++k) {
            dau[k + 1] = p[i] * nhat[k];
            rest[k + 1] = -(p[i] * nhat[k]);
        }
        if (i < n - 2) {
            const double gamma = sub[0] / sigma[i + 1];
            double eta[3];
            for (int k = 0; k < 3; ++k) eta[k] = sub[k + 1] / sigma[i + 1];
            boost(dau, eta, gamma);
            boost(rest, eta, gamma);
        }
        for (int mu = 0; mu < 4; ++mu) {
            p4[i + 1][mu] = dau[mu];
            sub[mu] = rest[mu];
        }
    }
    for (int mu = 0; mu < 4; ++mu) p4[0][mu] = sub[mu];

    if (parent4 != NULL) {
        const double gamma = parent4[0] / parent_mass;
        const double eta[3] = { parent4[1] / parent_mass, parent4[2] / parent_mass,
                                parent4[3] / parent_mass };
        for (int d = 0; d < n; ++d) boost(p4[d], eta, gamma);
    }
    return w;
}

/* Return codes shared in meaning (not in code) with the product library. */
#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_EKINEMATICS (-2)

static int check_args(double parent_mass, const double *masses, int n)
{
    if (n < 2 || n > ORACLE_NMAX || masses == NULL) return ORACLE_EINVAL;
    if (!(parent_mass > 0.0) || !isfinite(parent_mass)) return ORACLE_EINVAL;
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
        if (!(masses[i] >= 0.0) || !isfinite(masses[i])) return ORACLE_EINVAL;
        s += masses[i];
    }
    if (!(parent_mass - s > 0.0)) return ORACLE_EKINEMATICS;
    return ORACLE_OK;
}

/* Generate events e = 0..nevents-1 (global index event_offset + e).
 *   parent_p4     NULL, or one (E, px, py, pz) applied to every event;
 *   parent_soa    NULL, or per-event parents, component mu of event e at
 *                 parent_soa[mu * ld_parent + e];
 *   out           NULL, or SoA: component mu of daughter d of event e at
 *                 out[(4 d + mu) * ld + e];
 *   weights       NULL, or weights[e]. */
int oracle_generate(double parent_mass, const double *masses, int n,
                    const double *parent_p4, const double *parent_soa, uint64_t ld_parent,
                    uint64_t nevents, uint64_t seed, uint32_t stream_id, uint64_t event_offset,
                    double *out, uint64_t ld, double *weights)
{
    int st = check_args(parent_mass, masses, n);
    if (st != ORACLE_OK) return st;
    if (out != NULL && ld < nevents) return ORACLE_EINVAL;
    if (parent_soa != NULL && ld_parent < nevents) return ORACLE_EINVAL;
    double u[3 * ORACLE_NMAX];
    double p4[ORACLE_NMAX][4];
    for (uint64_t e = 0; e < nevents; ++e) {
        oracle_event_uniforms(seed, stream_id, event_offset + e, n, u);
        double parent[4];
        const double *pp = parent_p4;
        if (parent_soa != NULL) {
            for (int mu = 0; mu < 4; ++mu) parent[mu] = parent_soa[mu * ld_parent + e];
            pp = parent;
        }
        const double w = one_event(parent_mass, masses, n, pp, u, p4);
        if (weights != NULL) weights[e] = w;
        if (out != NULL)
            for (int d = 0; d < n; ++d)
                for (int mu = 0; mu < 4; ++mu) out[(uint64_t)(4 * d + mu) * ld + e] = p4[d][mu];
    }
    return ORACLE_OK;
}

/* Neumaier's compensated summation (improved Kahan-Babuska). */
typedef struct { double sum, comp; } nsum_t;

static void nsum_add(nsum_t *a, double x)
{
    const double t = a->sum + x;
    if (fabs(a->sum) >= fabs(x)) a->comp += (a->sum - t) + x;
    else a->comp += (x - t) + a->sum;
    a->sum = t;
}

/* Phase-space integral over events event_offset .. event_offset+nevents-1:
 *   mean  = (sum of weights) / n              (compensated sum),
 *   sigma = sqrt( sum (w - mean)^2 / ((n-1) n) )  (second pass, compensated),
 * i.e. the Monte Carlo estimate of R_N and its standard error. */
int oracle_integrate(double parent_mass, const double *masses, int n,
                     uint64_t nevents, uint64_t seed, uint32_t stream_id, uint64_t event_offset,
                     double *mean, double *sigma)
{
    int st = check_args(parent_mass, masses, n);
    if (st != ORACLE_OK) return st;
    if (nevents < 2 || mean == NULL || sigma == NULL) return ORACLE_EINVAL;
    double *w = (double *)malloc(sizeof(double) * nevents);
    if (w == NULL) return ORACLE_EINVAL;
    st = oracle_generate(parent_mass, masses, n, NULL, NULL, 0, nevents, seed, stream_id,
                         event_offset, NULL, 0, w);
    if (st == ORACLE_OK) {
        nsum_t s1 = { 0.0, 0.0 };
        for (uint64_t e = 0; e < nevents; ++e) nsum_add(&s1, w[e]);
        const double m = (s1.sum + s1.comp) / (double)nevents;
        nsum_t s2 = { 0.0, 0.0 };
        for (uint64_t e = 0; e < nevents; ++e) {
            const double d = w[e] - m;
            nsum_add(&s2, d * d);
        }
        const double var = (s2.sum + s2.comp) / (double)(nevents - 1);
        *mean = m;
        *sigma = sqrt(var / (double)nevents);
    }
    free(w);
    return st;
}

/* ---------------------------------------------------------------------- */
/* Unweighted samples (sec. 4.2 lists them next to weighted ones).  Plain   */
/* hit-or-miss: a trial event of weight w is kept with probability          */
/* min(1, w / w_max), so the kept events are distributed as phase space     */
/* itself (flat in the invariants) with unit weight.                        */
/* ---------------------------------------------------------------------- */

/* Number of Philox calls one event's uniforms use: ceil((3N-4)/2). */
int oracle_calls_per_event(int n)
{
    return (oracle_uniforms_per_event(n) + 1) / 2;
}

/* The acceptance uniform of global event g: words 0 and 1 of Philox call
 * j = oracle_calls_per_event(n) of the event's counter stream (the first call
 * its own uniforms do not use), converted like every other uniform. */
double oracle_accept_uniform(uint64_t seed, uint32_t stream_id, uint64_t g, int n)
{
    const uint32_t key[2] = { (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32) };
    const uint32_t ctr[4] = { (uint32_t)(g & 0xFFFFFFFFu), (uint32_t)(g >> 32),
                              (uint32_t)oracle_calls_per_event(n), stream_id };
    uint32_t words[4];
    oracle_philox4x32_10(ctr, key, words);
    uint64_t bits = ((uint64_t)words[1] << 32) | (uint64_t)words[0];
    uint64_t x = bits >> 12;
    return (double)(2 * x + 1) * 0x1p-53;
}

/* ---------------------------------------------------------------------- */
/* Model evaluation over phase space (sec. 4.2: "evaluation of model").    */
/* The model is a product of relativistic Breit-Wigner intensities in pair  */
/* invariant masses, |A|^2 = prod_k 1 / ((M_k^2 - s_k)^2 + M_k^2 G_k^2),    */
/* s_k = (p_i + p_j)^2 for the pair (i, j) of factor k; no factor is the    */
/* constant 1.  Each event contributes w |A|^2, so the mean is the integral */
/* of |A|^2 over phase space.                                               */
/* ---------------------------------------------------------------------- */

#define ORACLE_MAX_BW 4

/* s = (p_i + p_j)^2 = (E_i + E_j)^2 - |p_i + p_j|^2, components summed first. */
static double pair_mass_sq(const double a[4], const double b[4])
{
    const double e = a[0] + b[0], x = a[1] + b[1], y = a[2] + b[2], z = a[3] + b[3];
    return e * e - x * x - y * y - z * z;
}

static double model_intensity(double p4[][4], int n_bw, const int *pi, const int *pj, const double *mass,
                              const double *width)
{
    double a2 = 1.0;
    for (int k = 0; k < n_bw; ++k) {
        const double s = pair_mass_sq(p4[pi[k]], p4[pj[k]]);
        const double d = mass[k] * mass[k] - s;
        const double mg = mass[k] * width[k];
        a2 = a2 / (d * d + mg * mg);
    }
    return a2;
}

static int check_model(int n, int n_bw, const int *pi, const int *pj, const double *mass, const double *width)
{
    if (n_bw < 0 || n_bw > ORACLE_MAX_BW) return ORACLE_EINVAL;
    for (int k = 0; k < n_bw; ++k) {
        if (pi[k] < 0 || pj[k] >= n || pi[k] >= pj[k]) return ORACLE_EINVAL;
        if (!(mass[k] > 0.0) || !(width[k] > 0.0) || !isfinite(mass[k]) || !isfinite(width[k])) return ORACLE_EINVAL;
    }
    return ORACLE_OK;
}

/* Per-event values w |A|^2 of events e = 0..nevents-1 (parent at rest) into
 * values[e] (when not NULL), and their mean and standard error as in
 * oracle_integrate (compensated sum, second pass). */
int oracle_model_integrate(double parent_mass, const double *masses, int n, int n_bw, const int *pi,
                           const int *pj, const double *mass, const double *width, uint64_t nevents,
                           uint64_t seed, uint32_t stream_id, uint64_t event_offset, double *values,
                           double *mean, double *sigma)
{
    int st = check_args(parent_mass, masses, n);
    if (st != ORACLE_OK) return st;
    st = check_model(n, n_bw, pi, pj, mass, width);
    if (st != ORACLE_OK) return st;
    if (nevents < 2 || mean == NULL || sigma == NULL) return ORACLE_EINVAL;
    double *v = (double *)malloc(sizeof(double) * nevents);
    if (v == NULL) return ORACLE_EINVAL;
    double u[3 * ORACLE_NMAX];
    double p4[ORACLE_NMAX][4];
    for (uint64_t e = 0; e < nevents; ++e) {
        oracle_event_uniforms(seed, stream_id, event_offset + e, n, u);
        const double w = one_event(parent_mass, masses, n, NULL, u, p4);
        v[e] = w * model_intensity(p4, n_bw, pi, pj, mass, width);
        if (values != NULL) values[e] = v[e];
    }
    nsum_t s1 = { 0.0, 0.0 };
    for (uint64_t e = 0; e < nevents; ++e) nsum_add(&s1, v[e]);
    const double m = (s1.sum + s1.comp) / (double)nevents;
    nsum_t s2 = { 0.0, 0.0 };
    for (uint64_t e = 0; e < nevents; ++e) {
        const double d = v[e] - m;
        nsum_add(&s2, d * d);
    }
    *mean = m;
    *sigma = sqrt((s2.sum + s2.comp) / (double)(nevents - 1) / (double)nevents);
    free(v);
    return ORACLE_OK;
}

/* ---------------------------------------------------------------------- */
/* Unweighted (hit-or-miss) samples.  Trials e = 0..ntrials-1 (global index  */
/* event_offset + e) are the weighted events oracle_generate produces; the   */
/* trial's value is its weight w, or w |A|^2 for a model (parent at rest).   */
/* Trial e is kept when v * w_max < value, with v its acceptance uniform;    */
/* w_max == 0 takes the largest value of the trials (first pass).  Kept      */
/* events are written in trial order to out (SoA, capacity ld; kept events   */
/* past the capacity are counted, not written) and, when index is not NULL,  */
/* their global indices to index[0..].  counts[0] = number kept, counts[1] = */
/* number of trials whose value exceeds w_max (kept with probability 1, so   */
/* w_max did not bound them).  *w_max_used = the w_max applied.              */
/* ---------------------------------------------------------------------- */

typedef struct {
    int n_bw;
    const int *pi, *pj;
    const double *mass, *width;
} model_t;

static double trial_value(double parent_mass, const double *masses, int n, const double *parent_p4,
                          const model_t *model, const double *u, double p4[][4])
{
    const double w = one_event(parent_mass, masses, n, parent_p4, u, p4);
    if (model == NULL) return w;
    return w * model_intensity(p4, model->n_bw, model->pi, model->pj, model->mass, model->width);
}

static int unweight(double parent_mass, const double *masses, int n, const double *parent_p4, const model_t *model,
                    uint64_t ntrials, uint64_t seed, uint32_t stream_id, uint64_t event_offset, double w_max,
                    double *out, uint64_t ld, uint64_t *index, uint64_t counts[2], double *w_max_used)
{
    if (counts == NULL || !(w_max >= 0.0) || !isfinite(w_max)) return ORACLE_EINVAL;
    double u[3 * ORACLE_NMAX];
    double p4[ORACLE_NMAX][4];
    if (w_max == 0.0) {
        for (uint64_t e = 0; e < ntrials; ++e) {
            oracle_event_uniforms(seed, stream_id, event_offset + e, n, u);
            const double w = trial_value(parent_mass, masses, n, parent_p4, model, u, p4);
            if (w > w_max) w_max = w;
        }
    }
    uint64_t kept = 0, over = 0;
    for (uint64_t e = 0; e < ntrials; ++e) {
        const uint64_t g = event_offset + e;
        oracle_event_uniforms(seed, stream_id, g, n, u);
        const double w = trial_value(parent_mass, masses, n, parent_p4, model, u, p4);
        const double v = oracle_accept_uniform(seed, stream_id, g, n);
        if (w > w_max) ++over;
        if (v * w_max < w) {
            if (kept < ld) {
                if (out != NULL)
                    for (int d = 0; d < n; ++d)
                        for (int mu = 0; mu < 4; ++mu) out[(uint64_t)(4 * d + mu) * ld + kept] = p4[d][mu];
                if (index != NULL) index[kept] = g;
            }
            ++kept;
        }
    }
    counts[0] = kept;
    counts[1] = over;
    if (w_max_used != NULL) *w_max_used = w_max;
    return ORACLE_OK;
}

/* The trials' values are their weights (parent at rest, or the broadcast
 * parent_p4). */
int oracle_unweight(double parent_mass, const double *masses, int n, const double *parent_p4,
                    uint64_t ntrials, uint64_t seed, uint32_t stream_id, uint64_t event_offset,
                    double w_max, double *out, uint64_t ld, uint64_t *index, uint64_t counts[2],
                    double *w_max_used)
{
    int st = check_args(parent_mass, masses, n);
    if (st != ORACLE_OK) return st;
    return unweight(parent_mass, masses, n, parent_p4, NULL, ntrials, seed, stream_id, event_offset, w_max, out,
                    ld, index, counts, w_max_used);
}

/* The trials' values are w |A|^2 with the Breit-Wigner product above (parent
 * at rest): kept events follow the model's distribution over phase space. */
int oracle_unweight_model(double parent_mass, const double *masses, int n, int n_bw, const int *pi,
                          const int *pj, const double *mass, const double *width, uint64_t ntrials,
                          uint64_t seed, uint32_t stream_id, uint64_t event_offset, double w_max, double *out,
                          uint64_t ld, uint64_t *index, uint64_t counts[2], double *w_max_used)
{
    int st = check_args(parent_mass, masses, n);
    if (st != ORACLE_OK) return st;
    st = check_model(n, n_bw, pi, pj, mass, width);
    if (st != ORACLE_OK) return st;
    const model_t model = { n_bw, pi, pj, mass, width };
    return unweight(parent_mass, masses, n, NULL, &model, ntrials, seed, stream_id, event_offset, w_max, out, ld,
                    index, counts, w_max_used);
}

/* ---------------------------------------------------------------------- */
/* VEGAS importance sampling (Lepage, J. Comput. Phys. 27 (1978) 192; the   */
/* paper's sec. 4.1 uses it on a 10-dimensional Gaussian) and plain Monte   */
/* Carlo as its special case: one iteration on the uniform grid.            */
/*                                                                          */
/* Integrand: f(x) = prod_d exp(-(x_d - mu_d)^2 / (2 s_d^2)) / (s_d sqrt(2 pi))
/* over the box prod_d [lo_d, hi_d].  Grid: per dimension, K bins with edges */
/* g[d][0] = 0 < ... < g[d][K] = 1 in unit coordinates.  Sample i of        */
/* iteration t draws uniform u_d (uniform k of the counter stream           */
/* (i lo, i hi, j, t) under key seed, converted like the phase-space        */
/* uniforms); z = K u_d, bin b = floor(z), y = g[b] + (z - b)(g[b+1] - g[b]), */
/* x_d = lo_d + y (hi_d - lo_d); its value is f(x) J with                    */
/* J = prod_d K (g[b+1] - g[b]) (hi_d - lo_d).  The iteration's estimate is  */
/* the mean of the values with its standard error; the refinement histogram */
/* collects value^2 in each dimension's bin.                                */
/* ---------------------------------------------------------------------- */

#define ORACLE_VEGAS_DMAX 16
#define ORACLE_VEGAS_KMAX 128

static double gauss_factor(double x, double mu, double s)
{
    const double t = (x - mu) / s;
    return exp(-0.5 * t * t) / (s * 2.5066282746310002);   /* sqrt(2 pi) */
}

int oracle_vegas_iteration(int dim, int bins, const double *lo, const double *hi, const double *mu,
                           const double *sig, const double *grid, uint64_t calls, uint64_t seed,
                           uint32_t iteration, double *mean, double *sigma, double *hist, double *values)
{
    if (dim < 1 || dim > ORACLE_VEGAS_DMAX || bins < 1 || bins > ORACLE_VEGAS_KMAX || calls < 2) return ORACLE_EINVAL;
    if (mean == NULL || sigma == NULL || grid == NULL) return ORACLE_EINVAL;
    const uint32_t key[2] = { (uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32) };
    double *v = (double *)malloc(sizeof(double) * calls);
    if (v == NULL) return ORACLE_EINVAL;
    if (hist != NULL)
        for (int k = 0; k < dim * bins; ++k) hist[k] = 0.0;
    int binof[ORACLE_VEGAS_DMAX];
    for (uint64_t i = 0; i < calls; ++i) {
        uint32_t words[4 * ((ORACLE_VEGAS_DMAX + 1) / 2)];
        for (int j = 0; 2 * j < dim; ++j) {
            const uint32_t ctr[4] = { (uint32_t)(i & 0xFFFFFFFFu), (uint32_t)(i >> 32), (uint32_t)j, iteration };
            oracle_philox4x32_10(ctr, key, &words[4 * j]);
        }
        double val = 1.0;
        for (int d = 0; d < dim; ++d) {
            uint64_t bits = ((uint64_t)words[2 * d + 1] << 32) | (uint64_t)words[2 * d];
            const double u = (double)(2 * (bits >> 12) + 1) * 0x1p-53;
            const double z = u * (double)bins;
            int b = (int)z;
            if (b > bins - 1) b = bins - 1;
            const double *g = grid + d * (bins + 1);
            const double width = g[b + 1] - g[b];
            const double y = g[b] + (z - (double)b) * width;
            const double x = lo[d] + y * (hi[d] - lo[d]);
            val = val * gauss_factor(x, mu[d], sig[d]) * ((double)bins * width * (hi[d] - lo[d]));
            binof[d] = b;
        }
        v[i] = val;
        if (values != NULL) values[i] = val;
        if (hist != NULL)
            for (int d = 0; d < dim; ++d) hist[d * bins + binof[d]] += val * val;
    }
    nsum_t s1 = { 0.0, 0.0 };
    for (uint64_t i = 0; i < calls; ++i) nsum_add(&s1, v[i]);
    const double m = (s1.sum + s1.comp) / (double)calls;
    nsum_t s2 = { 0.0, 0.0 };
    for (uint64_t i = 0; i < calls; ++i) {
        const double dd = v[i] - m;
        nsum_add(&s2, dd * dd);
    }
    *mean = m;
    *sigma = sqrt((s2.sum + s2.comp) / (double)(calls - 1) / (double)calls);
    free(v);
    return ORACLE_OK;
}

/* Grid refinement of one VEGAS iteration, per dimension: the histogram h of
 * value^2 per bin is smoothed with its neighbours ((h[0]+h[1])/2, then
 * (h[k-1]+h[k]+h[k+1])/3, then (h[K-2]+h[K-1])/2); each bin gets the damped
 * importance r_k = ((1 - 1/R)/log R)^alpha with R = (sum of the smoothed h) /
 * smoothed h[k] (0 for an empty bin); the new edges cut the old grid, with
 * each old bin's share of importance spread evenly over its width, into K
 * pieces of equal importance.  Bins with no importance keep the grid. */
int oracle_vegas_refine(int dim, int bins, double *grid, const double *hist, double alpha)
{
    if (dim < 1 || dim > ORACLE_VEGAS_DMAX || bins < 2 || bins > ORACLE_VEGAS_KMAX || grid == NULL || hist == NULL)
        return ORACLE_EINVAL;
    double sm[ORACLE_VEGAS_KMAX], r[ORACLE_VEGAS_KMAX], edges[ORACLE_VEGAS_KMAX + 1];
    for (int d = 0; d < dim; ++d) {
        const double *h = hist + d * bins;
        double *g = grid + d * (bins + 1);
        double tot = 0.0;
        for (int k = 0; k < bins; ++k) {
            if (k == 0) sm[k] = (h[0] + h[1]) / 2.0;
            else if (k == bins - 1) sm[k] = (h[bins - 2] + h[bins - 1]) / 2.0;
            else sm[k] = (h[k - 1] + h[k] + h[k + 1]) / 3.0;
            tot += sm[k];
        }
        double rtot = 0.0;
        for (int k = 0; k < bins; ++k) {
            r[k] = 0.0;
            if (sm[k] > 0.0) {
                const double R = tot / sm[k];
                r[k] = R > 1.0 ? pow((1.0 - 1.0 / R) / log(R), alpha) : 1.0;
            }
            rtot += r[k];
        }
        if (!(rtot > 0.0)) continue;
        const double per = rtot / (double)bins;   /* importance per new bin */
        edges[0] = 0.0;
        int k = 0;            /* old bin being consumed */
        double left = r[0];   /* importance left in old bin k */
        for (int e = 1; e < bins; ++e) {
            double need = per;
            while (need > left && k < bins - 1) {
                need -= left;
                ++k;
                left = r[k];
            }
            left -= need;
            /* the new edge lies in old bin k, a fraction (r[k] - left)/r[k] into it */
            double frac = r[k] > 0.0 ? (r[k] - left) / r[k] : 1.0;
            if (frac < 0.0) frac = 0.0;   /* rounding of the running sums */
            if (frac > 1.0) frac = 1.0;
            edges[e] = g[k] + frac * (g[k + 1] - g[k]);
        }
        edges[bins] = 1.0;
        for (int e = 0; e <= bins; ++e) g[e] = edges[e];
    }
    return ORACLE_OK;
}

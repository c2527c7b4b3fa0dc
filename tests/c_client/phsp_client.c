/* A plain C client of the library: device memory from the HIP runtime, no
 * Python and no torch.  Generates n three-body events, integrates the same
 * events without storage, and prints what the calling test compares with the
 * oracle: the statuses, the fused integral, the synchronous integral, and the
 * weight and four-momenta of events 0 and n - 1.
 * Usage: phsp_client <n> <seed> */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "hydra_phsp.h"

#define MUST(x)                                                                          \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) {                                                          \
            fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 2;                                                                    \
        }                                                                                \
    } while (0)

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: phsp_client <n> <seed>\n");
        return 1;
    }
    const uint64_t n = strtoull(argv[1], NULL, 10);
    const uint64_t seed = strtoull(argv[2], NULL, 10);
    if (n < 2 || n > (1u << 24)) {
        fprintf(stderr, "n must be in [2, 2^24]\n");
        return 1;
    }
    const double M = 5.279;
    const double masses[3] = {3.097, 0.4937, 0.13957};
    const uint64_t ld = (n + 15) / 16 * 16; /* columns on 128-byte lines */
    double *out = NULL, *w = NULL, *stats = NULL;
    MUST(hipMalloc((void **)&out, sizeof(double) * 12 * ld));
    MUST(hipMalloc((void **)&w, sizeof(double) * n));
    MUST(hipMalloc((void **)&stats, sizeof(double) * HYDRA_PHSP_STATS));
    const int st_gen = hydra_phsp_generate(M, masses, 3, NULL, NULL, 0, n, seed, 0, 0, out, ld, w, stats, NULL);
    double mean = 0.0, sigma = 0.0;
    const int st_int = hydra_phsp_integrate(M, masses, 3, n, seed, 0, 0, &mean, &sigma, NULL);
    MUST(hipDeviceSynchronize());
    double s[HYDRA_PHSP_STATS], wf[2], p4[2][12];
    MUST(hipMemcpy(s, stats, sizeof(s), hipMemcpyDeviceToHost));
    MUST(hipMemcpy(&wf[0], w, sizeof(double), hipMemcpyDeviceToHost));
    MUST(hipMemcpy(&wf[1], w + (n - 1), sizeof(double), hipMemcpyDeviceToHost));
    for (int c = 0; c < 12; ++c) {
        MUST(hipMemcpy(&p4[0][c], out + (uint64_t)c * ld, sizeof(double), hipMemcpyDeviceToHost));
        MUST(hipMemcpy(&p4[1][c], out + (uint64_t)c * ld + (n - 1), sizeof(double), hipMemcpyDeviceToHost));
    }
    /* the same first stage with daughter 0 decaying to two muons, in one launch */
    const double mu2[2] = {0.1056583755, 0.1056583755};
    double *out2 = NULL, *w2 = NULL, *stats2 = NULL, *half = NULL;
    MUST(hipMalloc((void **)&out2, sizeof(double) * 8 * ld));
    MUST(hipMalloc((void **)&w2, sizeof(double) * ld));
    MUST(hipMalloc((void **)&stats2, sizeof(double) * HYDRA_PHSP_STATS));
    MUST(hipMalloc((void **)&half, sizeof(double) * 2 * HYDRA_PHSP_STATS));
    const int st_chain = hydra_phsp_generate_chain(M, masses, 3, 0, mu2, 2, n, seed, 0, 1, 0, out, ld, w, NULL, out2,
                                                   ld, w2, stats2, NULL);
    /* the integral in two pieces, merged on the host */
    const uint64_t cut = n / 2;
    const int st_a = hydra_phsp_integrate_async(M, masses, 3, cut, seed, 0, 0, half, NULL);
    const int st_b = hydra_phsp_integrate_async(M, masses, 3, n - cut, seed, 0, cut, half + HYDRA_PHSP_STATS, NULL);
    MUST(hipDeviceSynchronize());
    double h[2 * HYDRA_PHSP_STATS], merged[HYDRA_PHSP_STATS], q[2][8], wq[2];
    MUST(hipMemcpy(h, half, sizeof(h), hipMemcpyDeviceToHost));
    const int st_merge = hydra_phsp_stats_merge(h, h + HYDRA_PHSP_STATS, merged);
    MUST(hipMemcpy(&wq[0], w2, sizeof(double), hipMemcpyDeviceToHost));
    MUST(hipMemcpy(&wq[1], w2 + (n - 1), sizeof(double), hipMemcpyDeviceToHost));
    for (int c = 0; c < 8; ++c) {
        MUST(hipMemcpy(&q[0][c], out2 + (uint64_t)c * ld, sizeof(double), hipMemcpyDeviceToHost));
        MUST(hipMemcpy(&q[1][c], out2 + (uint64_t)c * ld + (n - 1), sizeof(double), hipMemcpyDeviceToHost));
    }
    printf("status %d %d\n", st_gen, st_int);
    printf("status2 %d %d %d %d\n", st_chain, st_a, st_b, st_merge);
    printf("merged %.17g %.17g %.17g %.17g\n", merged[0], merged[1], merged[2], merged[3]);
    for (int k = 0; k < 2; ++k) {
        printf("chain %llu %.17g", (unsigned long long)(k == 0 ? 0 : n - 1), wq[k]);
        for (int c = 0; c < 8; ++c) printf(" %.17g", q[k][c]);
        printf("\n");
    }
    MUST(hipFree(out2));
    MUST(hipFree(w2));
    MUST(hipFree(stats2));
    MUST(hipFree(half));
    printf("stats %.17g %.17g %.17g %.17g\n", s[0], s[1], s[2], s[3]);
    printf("integral %.17g %.17g\n", mean, sigma);
    for (int k = 0; k < 2; ++k) {
        printf("event %llu %.17g", (unsigned long long)(k == 0 ? 0 : n - 1), wf[k]);
        for (int c = 0; c < 12; ++c) printf(" %.17g", p4[k][c]);
        printf("\n");
    }
    MUST(hipFree(out));
    MUST(hipFree(w));
    MUST(hipFree(stats));
    return st_gen == HYDRA_PHSP_OK && st_int == HYDRA_PHSP_OK && st_chain == HYDRA_PHSP_OK && st_a == HYDRA_PHSP_OK &&
                   st_b == HYDRA_PHSP_OK && st_merge == HYDRA_PHSP_OK
               ? 0
               : 3;
}

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
    printf("status %d %d\n", st_gen, st_int);
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
    return st_gen == HYDRA_PHSP_OK && st_int == HYDRA_PHSP_OK ? 0 : 3;
}

/*
 * A C caller of libraysh, with no Python or torch in the process: it reads a
 * lens and a ray lattice from argv/stdin-free constants, shoots one FP64
 * map (Algorithm 1 of arXiv:1703.09707) through the C ABI, and prints the
 * number of binned rays and a checksum of the map; with a third argument it
 * also writes the map there (256 x 256 int32, row-major, native byte order).
 * Device memory comes from the HIP runtime directly.  Exit status: 0 on
 * success, 2 when raysh_init reports an error (for example when no GPU is
 * present), 1 otherwise.
 *
 * Usage: map_from_c <n_stars> <seed> [map_file]
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "raysh.h"

/* splitmix64: the star positions and masses are a deterministic function of
 * the seed, reproduced by the test that calls this program */
static uint64_t next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static double unit(uint64_t *s) { return (double)(next(s) >> 11) * (1.0 / 9007199254740992.0); }

int main(int argc, char **argv) {
    if (argc != 3 && argc != 4) {
        fprintf(stderr, "usage: %s <n_stars> <seed> [map_file]\n", argv[0]);
        return 1;
    }
    const int64_t n = atoll(argv[1]);
    uint64_t seed = strtoull(argv[2], NULL, 10);
    double *x = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *y = malloc(sizeof(double) * (n > 0 ? n : 1));
    double *m = malloc(sizeof(double) * (n > 0 ? n : 1));
    for (int64_t k = 0; k < n; ++k) {
        x[k] = 20.0 * unit(&seed) - 10.0;
        y[k] = 20.0 * unit(&seed) - 10.0;
        m[k] = 0.1 + 0.9 * unit(&seed);
    }
    raysh_lens lens = {0.1, 0.2, -0.05, n, x, y, m};
    raysh_ctx *ctx = NULL;
    int rc = raysh_init(&ctx, &lens, 0, NULL);
    free(x);
    free(y);
    free(m);
    if (rc != RAYSH_OK) {
        printf("raysh_init: code %d: %s\n", rc, raysh_last_error());
        return 2;
    }
    const raysh_rays rays = {-12.0, -12.0, 24.0 / 1024, 24.0 / 1024, 1024, 1024, 0, 0};
    const raysh_pixels pix = {-5.0, -5.0, 10.0 / 256, 10.0 / 256, 256, 256};
    int32_t *counts = NULL;
    if (hipMalloc((void **)&counts, sizeof(int32_t) * 256 * 256) != hipSuccess ||
        hipMemset(counts, 0, sizeof(int32_t) * 256 * 256) != hipSuccess) {
        printf("device allocation failed\n");
        raysh_free(ctx);
        return 1;
    }
    uint64_t binned = 0;
    rc = raysh_map(ctx, &rays, &pix, RAYSH_FP64, counts, &binned);
    if (rc != RAYSH_OK) {
        printf("raysh_map: code %d: %s\n", rc, raysh_last_error());
        return 1;
    }
    int32_t *host = malloc(sizeof(int32_t) * 256 * 256);
    if (hipMemcpy(host, counts, sizeof(int32_t) * 256 * 256, hipMemcpyDeviceToHost) != hipSuccess) {
        printf("copy failed\n");
        return 1;
    }
    uint64_t sum = 0, weighted = 0;
    for (int i = 0; i < 256 * 256; ++i) {
        sum += (uint64_t)host[i];
        weighted += (uint64_t)host[i] * (uint64_t)(i + 1);
    }
    printf("binned %llu sum %llu weighted %llu\n", (unsigned long long)binned, (unsigned long long)sum,
           (unsigned long long)weighted);
    if (argc == 4) {
        FILE *f = fopen(argv[3], "wb");
        if (!f || fwrite(host, sizeof(int32_t), 256 * 256, f) != 256 * 256 || fclose(f) != 0) {
            printf("cannot write %s\n", argv[3]);
            return 1;
        }
    }
    free(host);
    (void)hipFree(counts);
    return raysh_free(ctx) == RAYSH_OK ? 0 : 1;
}

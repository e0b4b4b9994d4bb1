/*
 * Drives the CPU oracle through every entry point on small inputs so that an
 * AddressSanitizer / UndefinedBehaviorSanitizer build can check it (test
 * infrastructure: tests/test_sanitizers.py compiles and runs it).  Inputs:
 * the depth map of a fronto-parallel plane seen head-on, with a hole and a
 * ragged image size; a raycast from the same camera; marching cubes, export,
 * eviction and re-import of the fused blocks.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "oracle.h"

int main(void)
{
    const int32_t dims[3] = {64, 48, 40};
    const double origin[3] = {-0.16, -0.12, 0.3};
    const double vs = 0.005;
    orc_volume *v = orc_create(dims, vs, origin, 4.0, 1e-4, 4096);
    if (!v) return 2;
    const int W = 37, H = 29;
    float *depth = malloc(sizeof(float) * W * H);
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) depth[j * W + i] = (i == 5 && j == 7) ? 0.0f : 0.4f + 0.001f * (float)i;
    const double K[4] = {40.0, 40.0, 18.0, 14.0};
    const double pose[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
    orc_stats st;
    for (int f = 0; f < 3; ++f)
        if (orc_integrate(v, depth, W, H, K, pose, ORC_NOISE_QUADRATIC, 0.0015, NULL, &st) != ORC_OK) return 3;
    orc_set_threads(v, 2);
    if (orc_integrate(v, depth, W, H, K, pose, ORC_NOISE_CONSTANT, 0.01, NULL, &st) != ORC_OK) return 4;
    const int64_t n = (int64_t)W * H;
    double *vert = calloc(4 * n, sizeof(double)), *nrm = calloc(4 * n, sizeof(double));
    int32_t *flags = calloc(n, sizeof(int32_t));
    orc_raycast(v, W, H, K, pose, NULL, n, vert, nrm, flags, 1);
    int hits = 0;
    for (int64_t k = 0; k < n; ++k) hits += (flags[k] & ORC_HIT) != 0;
    int64_t ntri = orc_marching_cubes(v, NULL, NULL, NULL, 0);
    int64_t *vid = malloc(sizeof(int64_t) * 3 * (ntri + 1));
    double *t = malloc(sizeof(double) * 3 * (ntri + 1)), *pos = malloc(sizeof(double) * 9 * (ntri + 1));
    if (orc_marching_cubes(v, vid, t, pos, ntri) != ntri) return 5;
    int32_t edges[3 * ORC_MC_MAX_TRIS];
    for (int c = 0; c < 256; ++c)
        if (orc_mc_case(c, edges) < 0) return 6;
    const int64_t nb = orc_block_count(v);
    int32_t *keys = malloc(sizeof(int32_t) * 3 * nb);
    double *T = malloc(sizeof(double) * 512 * nb), *P = malloc(sizeof(double) * 512 * nb);
    orc_export(v, keys, T, P, nb);
    const int32_t lo[3] = {0, 0, 0}, hi[3] = {3, 5, 4};
    int64_t ne = orc_evict(v, lo, hi, keys, T, P, nb);
    if (ne < 0) return 7;
    for (int64_t b = 0; b < ne; ++b)
        if (orc_set_block(v, keys + 3 * b, T + 512 * b, P + 512 * b) != ORC_OK) return 8;
    orc_set_rule(v, ORC_RULE_WEIGHTED, ORC_WEIGHT_INV_VARIANCE, 1.0, 64.0);
    if (orc_integrate(v, depth, W, H, K, pose, ORC_NOISE_QUADRATIC, 0.0015, NULL, &st) != ORC_OK) return 9;
    printf("blocks %lld hits %d triangles %lld evicted %lld\n", (long long)nb, hits, (long long)ntri, (long long)ne);
    free(depth); free(vert); free(nrm); free(flags); free(vid); free(t); free(pos); free(keys); free(T); free(P);
    orc_destroy(v);
    return (hits > 0 && ntri > 0 && ne > 0) ? 0 : 10;
}

// Per-pixel features of the learned noise model, computed per 16x16 pixel
// tile with a 16-pixel halo staged in LDS.
//
//   f0 = D (metres)
//   f1 = |cos| between the view ray and the surface normal; the normal is the
//        cross product of the central differences of the back-projected
//        neighbours along i and j (all four neighbours valid, pixel not on the
//        image border); computed in double
//   f2 = min(Euclidean distance to the nearest depth discontinuity, 16) / 16;
//        a discontinuity is a valid pixel with an in-image 4-neighbour that is
//        invalid or differs by more than 5 % of its depth.  Exact separable
//        transform inside the 33x33 window: min over dy of dy^2 + g(dy)^2,
//        g = nearest discontinuity along the row (from the row's bit mask)
//   f3 = radial pixel distance to the principal point / fx
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace tsdf {

constexpr int kFeatTile = 16;
constexpr int kFeatHalo = 16;
constexpr int kFeatRegion = kFeatTile + 2 * kFeatHalo;   // 48 (discontinuity region)
constexpr int kFeatDepth = kFeatRegion + 2;              // 50 (depth incl. the neighbour ring)

struct FeatLds {
    float dep[kFeatDepth + 2][kFeatDepth + 1];   // NaN = outside the image, 0 = no measurement; the last
                                                 // two rows take the staging loop's partial round
    unsigned long long disc[kFeatRegion];    // discontinuities of each region row, bit c = column c
    uint8_t g[kFeatRegion][kFeatTile];       // row distance to the nearest discontinuity (17 = none)
};

// All 256 threads of the workgroup call this (workgroup barriers inside).
// Thread t handles pixel (i0 + t % 16, j0 + t / 16).  Returns validity.
__device__ inline bool tile_features(FeatLds &L, const float *__restrict__ depth, int W, int H, double fx, double fy,
                                     double cx, double cy, int i0, int j0, int tid, float f[4])
{
    const float kOut = __uint_as_float(0x7fc00000u);   // quiet NaN: outside the image
    // every load of the thread is issued before the first LDS store (one
    // memory round trip, not one per element); the index is clamped into the
    // image so that each load is in bounds, and the value replaced outside it
    constexpr int kN = kFeatDepth * kFeatDepth, kPer = (kN + 255) / 256;
    static_assert(kPer * 256 <= (kFeatDepth + 2) * kFeatDepth, "the padding rows take the partial round");
    float d[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int k = min(tid + 256 * q, kN - 1);
        const int r = k / kFeatDepth, c = k % kFeatDepth;
        const int jj = j0 - kFeatHalo - 1 + r, ii = i0 - kFeatHalo - 1 + c;
        d[q] = depth[(size_t)min(max(jj, 0), H - 1) * W + min(max(ii, 0), W - 1)];
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int k = tid + 256 * q;   // below kPer * 256 <= (kFeatDepth + 2) * kFeatDepth
        const int r = k / kFeatDepth, c = k % kFeatDepth;
        const int jj = j0 - kFeatHalo - 1 + r, ii = i0 - kFeatHalo - 1 + c;
        float x = d[q];
        if (!(x > 0.0f) || !isfinite(x)) x = 0.0f;
        L.dep[r][c] = (ii >= 0 && jj >= 0 && ii < W && jj < H) ? x : kOut;
    }
    __syncthreads();
    // discontinuity bits: wavefront w takes rows w, w + 4, ..., lane c < 48 one
    // column, and the row's ballot is its bit mask
    // (the tests are combined with non-short-circuit operators, so that a row
    // is straight-line code; lanes 48..63 read an in-bounds column and drop it)
    const int lane = tid & 63;
    const int cl = min(lane, kFeatRegion - 1);
#pragma unroll
    for (int r0 = 0; r0 < kFeatRegion; r0 += 12) {
        const int r = r0 + 3 * (tid >> 6);
        float D[3], nb[3][4];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            D[e] = L.dep[r + e + 1][cl + 1];
            nb[e][0] = L.dep[r + e + 1][cl + 2];
            nb[e][1] = L.dep[r + e + 1][cl];
            nb[e][2] = L.dep[r + e + 2][cl + 1];
            nb[e][3] = L.dep[r + e][cl + 1];
        }
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const double Dd = (double)D[e], thr = 0.05 * Dd;
            bool any = false;
#pragma unroll
            for (int q = 0; q < 4; ++q)   // a neighbour outside the image (NaN) does not count
                any |= !isnan(nb[e][q]) & (!(nb[e][q] > 0.0f) | (fabs((double)nb[e][q] - Dd) > thr));
            const bool dsc = (lane < kFeatRegion) & (D[e] > 0.0f) & any;   // D > 0 is false for NaN and 0
            const unsigned long long m = __ballot(dsc);
            if (lane == 0) L.disc[r + e] = m;
        }
    }
    __syncthreads();
    // distance along the row to the nearest discontinuity within 16 columns:
    // the lowest set bit at or right of the column, the highest at or left of it
    for (int k = tid; k < kFeatRegion * kFeatTile; k += 256) {
        const int r = k / kFeatTile, pos = k % kFeatTile + kFeatHalo;
        const unsigned long long m = L.disc[r];
        const unsigned long long right = m >> pos, left = m << (63 - pos);
        const int dr = right ? __builtin_ctzll(right) : 64, dl = left ? __builtin_clzll(left) : 64;
        const int best = min(dl, dr);
        L.g[r][k % kFeatTile] = (uint8_t)(best > kFeatHalo ? kFeatHalo + 1 : best);
    }
    __syncthreads();
    const int ti = tid % kFeatTile, tj = tid / kFeatTile;
    const int i = i0 + ti, j = j0 + tj;
    const float D = L.dep[tj + kFeatHalo + 1][ti + kFeatHalo + 1];
    f[0] = f[1] = f[2] = f[3] = 0.0f;
    if (!(D > 0.0f)) return false;
    int d2 = 1 << 30;
    for (int dy = -kFeatHalo; dy <= kFeatHalo; ++dy) {
        const int gx = L.g[tj + kFeatHalo + dy][ti];
        d2 = min(d2, dy * dy + gx * gx);
    }
    // pixel offsets scaled by 1/f (products with the reciprocals: equal to the
    // quotients to an ulp)
    const double ifx = 1.0 / fx, ify = 1.0 / fy;
    f[0] = D;
    f[2] = fminf(sqrtf((float)d2), 16.0f) / 16.0f;
    f[3] = (float)(sqrt((i - cx) * (i - cx) + (j - cy) * (j - cy)) * ifx);
    if (i < 1 || j < 1 || i >= W - 1 || j >= H - 1) return false;
    const float Dl = L.dep[tj + kFeatHalo + 1][ti + kFeatHalo], Dr = L.dep[tj + kFeatHalo + 1][ti + kFeatHalo + 2];
    const float Du = L.dep[tj + kFeatHalo][ti + kFeatHalo + 1], Dd = L.dep[tj + kFeatHalo + 2][ti + kFeatHalo + 1];
    if (!(Dl > 0.0f && Dr > 0.0f && Du > 0.0f && Dd > 0.0f)) return false;
    const double ax = (i + 1 - cx) * ifx * Dr - (i - 1 - cx) * ifx * Dl;
    const double ay = (j - cy) * ify * Dr - (j - cy) * ify * Dl;
    const double az = (double)Dr - (double)Dl;
    const double bx = (i - cx) * ifx * Dd - (i - cx) * ifx * Du;
    const double by = (j + 1 - cy) * ify * Dd - (j - 1 - cy) * ify * Du;
    const double bz = (double)Dd - (double)Du;
    const double nx = ay * bz - az * by, ny = az * bx - ax * bz, nz = ax * by - ay * bx;
    const double nl = sqrt(nx * nx + ny * ny + nz * nz);
    const double rx = (i - cx) * ifx, ry = (j - cy) * ify;
    const double rl = sqrt(rx * rx + ry * ry + 1.0);
    if (!(nl > 0.0)) return false;
    f[1] = (float)(fabs(nx * rx + ny * ry + nz) / (nl * rl));
    return true;
}

}  // namespace tsdf

// Device bodies of frame preparation and block fusion, shared by the
// single-volume kernels (fuse.hip) and the batched multi-scene kernels
// (batch.hip).  See fuse.hip for the method.
#pragma once

#include <type_traits>

#include "tsdf_internal.h"
#include "mlp_device.h"
#include "mlp_features.h"

namespace tsdf {

// Per-frame counter reset; thread t < kCtrLanes clears lane t.
__device__ __forceinline__ void frame_begin_body(DeviceState *st, Counters *ctr, int t)
{
    if (t < kCtrLanes)
        for (int c = 0; c < CTR_N; ++c) ctr->frame[t][c] = 0;
    if (t == 0) {
        st->cand_count = 0;
        st->frames += 1;
    }
}

// ---------------------------------------------------------------- prep

constexpr int kTile = 16;             // 16x16 pixels per workgroup
constexpr int kLdsSet = 2048;         // LDS hash set of block keys
constexpr int kLdsList = 1024;        // unique keys held for the global pass
constexpr int kSubRanges = 2;         // depth sub-intervals of a pixel's frustum cell

// Marks `key` as a candidate of this frame; the first marker appends it to
// the candidate list.  Used, one lane at a time, for keys that did not fit
// the LDS set; the tile's other keys are appended together (prep_body).
__device__ inline void global_candidate_lane(const VolumeView &v, uint32_t key, int bx, int by, int bz)
{
    uint64_t b = block_linear(v, bx, by, bz);
    uint32_t bit = 1u << (b & 31);
    uint32_t old = atomicOr(&v.cand_bits[b >> 5], bit);
    if (old & bit) return;
    uint32_t idx = atomicAdd(&v.state->cand_count, 1u);
    if (idx < v.max_candidates) {
        v.cand_list[idx] = key;
    } else {
        atomicOr(&v.state->status, (uint32_t)TSDF_FLAG_CAND_FULL);
        atomicAnd(&v.cand_bits[b >> 5], ~bit);
    }
}

__device__ inline float measurement_variance(const NoiseParams &noise, float D, float inv_delta)
{
    if (noise.kind == TSDF_NOISE_CONSTANT) return noise.coeff;
    float r = noise.coeff * D * D * inv_delta;   // sigma / delta
    return r * r;
}

struct PrepCandLds {
    uint32_t set[kLdsSet];
    uint32_t list[kLdsList];
};
// MLP mode: the feature tile and the network scratch are dead before the
// candidate pass starts, so the three share one region.
struct PrepMlpLds {
    union {
        PrepCandLds cand;
        FeatLds feat;
        MlpInferLds wave[4];
    } u;
    MlpParamsLds P;
};

// One 16x16 pixel tile (tx, ty) of one frame.  Called by all 256 threads.
template <bool kMlp>
__device__ __forceinline__ void prep_body(const VolumeView &v, const float *__restrict__ depth, const Camera &cam,
                                          const NoiseParams &noise, int tx, int ty)
{
    using Lds = typename std::conditional<kMlp, PrepMlpLds, PrepCandLds>::type;
    __shared__ Lds lds;
    __shared__ uint32_t n_list;
    const int tid = threadIdx.x;
    const int i = tx * kTile + (tid & (kTile - 1));
    const int j = ty * kTile + (tid / kTile);
    const bool in_image = i < cam.width && j < cam.height;
    float D = in_image ? depth[(size_t)j * cam.width + i] : 0.0f;
    const bool valid = in_image && D > 0.0f && isfinite(D);
    // a tile without a valid pixel (background) only clears its pixel map
    if (!__syncthreads_or(valid)) {
        if (in_image) v.pixmap[(size_t)j * cam.width + i] = make_float2(0.0f, 0.0f);
        return;
    }
    const float inv_delta_f = (float)v.inv_delta;
    float ph = valid ? measurement_variance(noise, D, inv_delta_f) : 0.0f;
    PrepCandLds *cand;
    if constexpr (kMlp) {
        // learned variance: features of this tile, then the network (matrix cores)
        PrepMlpLds &L = lds;
        mlp_stage_params(L.P, (const uint16_t *)noise.mlp, tid, 256);
        float f[4];
        const bool fok = tile_features(L.u.feat, depth, cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy,
                                       tx * kTile, ty * kTile, tid, f);
        __syncthreads();
        const float s = mlp_infer_wave(L.P, (const uint16_t *)noise.mlp, L.u.wave[tid >> 6], f, tid & 63);
        if (valid && fok) {
            const float pl = __expf(s) * inv_delta_f * inv_delta_f;
            ph = fminf(fmaxf(pl, ph * 0.018315639f), ph * 54.59815f);   // [p_q e^-4, p_q e^4]
        }
        __syncthreads();
        cand = &L.u.cand;
    } else {
        cand = &lds;
    }
    uint32_t *set = cand->set;
    uint32_t *list = cand->list;
    for (int k = tid; k < kLdsSet; k += 256) set[k] = kEmptyKey;
    if (tid == 0) n_list = 0;
    if (in_image) v.pixmap[(size_t)j * cam.width + i] = make_float2(valid ? D : 0.0f, ph);
    __syncthreads();

    if (valid) {
        // The frustum cell (pixel square x [D - delta, D + delta]) is cut into
        // kSubRanges depth slices; each slice's world box gives candidate
        // blocks (those whose voxel centres the box may contain).
        const double z0 = fmax((double)D - v.delta, 0.0), z1 = (double)D + v.delta;
        const double ul = (i - 0.5 - cam.cx) / cam.fx, uh = (i + 0.5 - cam.cx) / cam.fx;
        const double vl = (j - 0.5 - cam.cy) / cam.fy, vh = (j + 0.5 - cam.cy) / cam.fy;
        // A slice [za, zb] is spanned by the points z * d + t, d the rotated
        // direction of a point of the pixel square at unit depth: as z > 0,
        // its box per axis is the span of z * [dmin, dmax] over the two depths,
        // [dmin, dmax] the range of d (separable in the square's two sides).
        // Kept in grid units; the pad of 1 % of a voxel covers the rounding.
        const double pad = 0.01 * v.vs;
        double emin[3], emax[3], cmin[3], cmax[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double r0 = cam.R[3 * a], r1 = cam.R[3 * a + 1], r2 = cam.R[3 * a + 2];
            const double p0 = r0 * ul, p1 = r0 * uh, q0 = r1 * vl, q1 = r1 * vh;
            emin[a] = (fmin(p0, p1) + fmin(q0, q1) + r2) * v.inv_vs;
            emax[a] = (fmax(p0, p1) + fmax(q0, q1) + r2) * v.inv_vs;
            cmin[a] = (cam.t[a] - pad - v.origin[a]) * v.inv_vs - 0.5;
            cmax[a] = (cam.t[a] + pad - v.origin[a]) * v.inv_vs - 0.5;
        }
        for (int sr = 0; sr < kSubRanges; ++sr) {
            const double za = z0 + (z1 - z0) * sr / kSubRanges;
            const double zb = (sr == kSubRanges - 1) ? z1 : z0 + (z1 - z0) * (sr + 1) / kSubRanges;
            int b0[3], b1[3];
            bool empty = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double g0 = ceil(fmin(za * emin[a], zb * emin[a]) + cmin[a]);
                double g1 = floor(fmax(za * emax[a], zb * emax[a]) + cmax[a]);
                g0 = fmax(g0, 0.0);
                g1 = fmin(g1, (double)(v.dims[a] - 1));
                empty |= !(g0 <= g1);
                b0[a] = empty ? 0 : (int)g0 >> 3;
                b1[a] = empty ? -1 : (int)g1 >> 3;
            }
            if (empty) continue;
            for (int bz = b0[2]; bz <= b1[2]; ++bz)
                for (int by = b0[1]; by <= b1[1]; ++by)
                    for (int bx = b0[0]; bx <= b1[0]; ++bx) {
                        const uint32_t key = pack_key(bx, by, bz);
                        uint32_t h = hash_key(key) & (kLdsSet - 1);
                        bool placed = false;
                        for (int p = 0; p < 64; ++p) {
                            uint32_t prev = atomicCAS(&set[h], kEmptyKey, key);
                            if (prev == kEmptyKey) {
                                uint32_t slot = atomicAdd(&n_list, 1u);
                                if (slot < (uint32_t)kLdsList) {
                                    list[slot] = key;
                                    placed = true;
                                }
                                break;
                            }
                            if (prev == key) {
                                placed = true;
                                break;
                            }
                            h = (h + 1) & (kLdsSet - 1);
                        }
                        // LDS set or list exhausted: go straight to the frame-wide dedup
                        if (!placed) global_candidate_lane(v, key, bx, by, bz);
                    }
        }
    }
    __syncthreads();
    const uint32_t n = min(n_list, (uint32_t)kLdsList);
    if (n == 0) return;
    // Keys this tile is first to mark are compacted into the (now unused)
    // set and appended with one counter update per tile: a counter update
    // per wavefront makes every tile of the frame queue on one address.
    __shared__ uint32_t n_fresh, base;
    if (tid == 0) n_fresh = 0;
    __syncthreads();
    for (uint32_t k = tid; k < n; k += 256) {
        const uint32_t key = list[k];
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        const uint64_t b = block_linear(v, bx, by, bz);
        const uint32_t bit = 1u << (b & 31);
        if (!(atomicOr(&v.cand_bits[b >> 5], bit) & bit)) set[atomicAdd(&n_fresh, 1u)] = key;
    }
    __syncthreads();
    if (tid == 0 && n_fresh) base = atomicAdd(&v.state->cand_count, n_fresh);
    __syncthreads();
    for (uint32_t k = tid; k < n_fresh; k += 256) {
        const uint32_t key = set[k];
        const uint32_t idx = base + k;
        if (idx < v.max_candidates) {
            v.cand_list[idx] = key;
        } else {
            int bx, by, bz;
            unpack_key(key, bx, by, bz);
            const uint64_t b = block_linear(v, bx, by, bz);
            atomicOr(&v.state->status, (uint32_t)TSDF_FLAG_CAND_FULL);
            atomicAnd(&v.cand_bits[b >> 5], ~(1u << (b & 31)));
        }
    }
}

// ---------------------------------------------------------------- fuse

// Per-frame constants of the voxel projection.  Along a lane's voxel column
// (grid z) the camera coordinates advance by R^T (0, 0, voxel): the decisions
// start from the exact coordinates of the column's first voxel plus z times
// that step, which differs from the defined double expression by at most
// `err` metres; the decisions below are taken only where that difference
// cannot change them, otherwise the defined expression is evaluated.
struct FuseCam {
    double sx, sy, sz;   // camera-frame step per voxel along grid z
    double err;          // bound on |approximate - defined| camera coordinate
    double ceu, cev;     // pixel margin: r * ce + cr, r = 1 / z_c
    double cru, crv;
    double thr_s;        // |s| within thr_s of delta: decided by the defined expression
};

__host__ __device__ inline FuseCam make_fuse_cam(const VolumeView &v, const Camera &cam)
{
    FuseCam f;
    f.sx = cam.R[6] * v.vs;
    f.sy = cam.R[7] * v.vs;
    f.sz = cam.R[8] * v.vs;
    // magnitude bound of every intermediate (positions, differences, camera coordinates)
    double m = 0.0, mt = 0.0;
    for (int a = 0; a < 3; ++a) {
        m = fmax(m, fabs(v.origin[a]) + (double)v.dims[a] * v.vs);
        mt = fmax(mt, fabs(cam.t[a]));
    }
    const double M = 3.0 * (m + mt) + 1.0;
    const double ulp = 1.1102230246251565e-16;   // 2^-53
    f.err = 192.0 * ulp * M;
    // |u~ - u| <= (fx + |a_u|) err / z_c + rounding, with |a_u| <= W + 2 + |c_x|
    // wherever the decision can be near a pixel boundary inside the image
    const double au = cam.width + 2.0 + fabs(cam.cx), av = cam.height + 2.0 + fabs(cam.cy);
    f.ceu = 2.0 * f.err * (cam.fx + au);
    f.cev = 2.0 * f.err * (cam.fy + av);
    f.cru = 64.0 * ulp * au + 1e-300;
    f.crv = 64.0 * ulp * av + 1e-300;
    f.thr_s = 4.0 * f.err + 64.0 * ulp * M;
    return f;
}

// Nearest-pixel index from approximate camera coordinates (within fc.err of
// the defined ones): the linear pixel index, -1 outside the image or behind
// the camera, -2 when only the defined expression can decide.
__device__ __forceinline__ int pixel_filter(const Camera &cam, const FuseCam &fc, double xc, double yc, double zc)
{
    if (!(zc > 2.0 * fc.err)) return zc < -2.0 * fc.err ? -1 : -2;
    double r = __builtin_amdgcn_rcp(zc);
    r = fma(r, fma(-zc, r, 1.0), r);   // two Newton steps: r = 1/z_c to a few ulp
    r = fma(r, fma(-zc, r, 1.0), r);
    const double tu = fma(cam.fx * xc, r, cam.cx + 0.5), tv = fma(cam.fy * yc, r, cam.cy + 0.5);
    const double fu = floor(tu), fv = floor(tv);
    const double du = tu - fu, dv = tv - fv;
    const double eu = fma(r, fc.ceu, fc.cru), ev = fma(r, fc.cev, fc.crv);
    if (!(du > eu && du < 1.0 - eu && dv > ev && dv < 1.0 - ev)) return -2;
    if (!(fu >= 0.0 && fu < (double)cam.width && fv >= 0.0 && fv < (double)cam.height)) return -1;
    return (int)fv * cam.width + (int)fu;
}

// The defined double expression: i = floor(fx x_c / z_c + cx + 1/2), same for j.
// Scalars by value: a reference would force the kernel's camera into scratch.
__device__ __forceinline__ int pixel_exact(double fx, double fy, double cx, double cy, int width, int height,
                                        double xc, double yc, double zc)
{
#pragma clang fp contract(off)
    const double u = fx * xc / zc + cx;
    const double w = fy * yc / zc + cy;
    const double fu = floor(u + 0.5), fw = floor(w + 0.5);
    if (!(fu >= 0.0 && fu < (double)width && fw >= 0.0 && fw < (double)height)) return -1;
    return (int)fw * width + (int)fu;
}

__device__ __forceinline__ void kalman(float &T, float &P, float Tk, float pk, float q)
{
    // Algorithm 3 in normalised units; chi is any |T| > 1
    if (fabsf(T) > 1.0f) {
        T = Tk;
        P = pk;
    } else {
        // K = P / (P + p_k); the new variance (1 - K) P is formed as K p_k,
        // which is the same quantity without the cancellation in 1 - K
        P = P + q;
        const float K = P * __builtin_amdgcn_rcpf(P + pk);
        T = T + K * (Tk - T);
        P = K * pk;
    }
    if (fabsf(T) > 1.0f) T = kChi;
}

// Algorithm 1: T <- (1 - w) T + w T_k, evaluated as T + w (T_k - T) (a first
// measurement sets T = T_k).  The fused forms are written out so that every
// kernel that inlines these rules rounds them the same way.
__device__ __forceinline__ void running_mean(float &T, float Tk, float w)
{
    T = fabsf(T) > 1.0f ? Tk : fmaf(w, Tk - T, T);
    if (fabsf(T) > 1.0f) T = kChi;
}

// Algorithm 2: the weighted mean with weight sum W (kept in P's place),
// capped at w_max; a first measurement sets T = T_k, W = w_k.
__device__ __forceinline__ void weighted_mean(float &T, float &W, float Tk, float wk, float w_max)
{
    if (fabsf(T) > 1.0f) {
        T = Tk;
        W = wk;
    } else {
        T = fmaf(W, T, wk * Tk) * __builtin_amdgcn_rcpf(W + wk);
        W = fminf(W + wk, w_max);
    }
    if (fabsf(T) > 1.0f) T = kChi;
}

// The volume's update rule on one voxel with a measurement (the rule is a
// template argument so that each rule's loop is compiled on its own).
template <int kRule>
__device__ __forceinline__ void update_voxel(const VolumeView &v, float &T, float &P, float Tk, float pk)
{
    if constexpr (kRule == TSDF_RULE_KALMAN) {
        kalman(T, P, Tk, pk, v.q_hat);
    } else if constexpr (kRule == TSDF_RULE_RUNNING) {
        running_mean(T, Tk, v.w);
    } else {
        weighted_mean(T, P, Tk, v.weight_kind == TSDF_WEIGHT_INV_VARIANCE ? __builtin_amdgcn_rcpf(pk) : v.w,
                      v.w_max);
    }
}

// What P holds after a voxel's first measurement under the volume's rule.
__device__ __forceinline__ float first_p(const VolumeView &v, float pk)
{
    if (v.rule == TSDF_RULE_KALMAN) return pk;
    if (v.rule == TSDF_RULE_RUNNING) return 0.0f;
    return v.weight_kind == TSDF_WEIGHT_INV_VARIANCE ? __builtin_amdgcn_rcpf(pk) : v.w;
}

template <typename S>
__device__ __forceinline__ float load_s(const S *p);
template <>
__device__ __forceinline__ float load_s<float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float load_s<__half>(const __half *p) { return __half2float(*p); }
template <typename S>
__device__ __forceinline__ void store_s(S *p, float x);
template <>
__device__ __forceinline__ void store_s<float>(float *p, float x) { *p = x; }
template <>
__device__ __forceinline__ void store_s<__half>(__half *p, float x) { *p = __float2half_rn(x); }

// A value as it reads back from storage of type S.
template <typename S>
__device__ __forceinline__ float stored_value(float x);
template <>
__device__ __forceinline__ float stored_value<float>(float x) { return x; }
template <>
__device__ __forceinline__ float stored_value<__half>(float x) { return __half2float(__float2half_rn(x)); }

// Workgroups (of four wavefronts) of the persistent fusion grid.
constexpr uint32_t kFuseGrid = 2560;

// P as it goes to storage: FP16 cannot hold an Algorithm 2 weight sum above
// 65504, so it is clamped there (variances never come near it).
template <typename S>
__device__ __forceinline__ float stored_weight(float p);
template <>
__device__ __forceinline__ float stored_weight<float>(float p) { return p; }
template <>
__device__ __forceinline__ float stored_weight<__half>(float p) { return fminf(p, 65504.0f); }

// Event counts a wavefront accumulates over the candidates it processes.
struct FuseAcc {
    uint32_t upd = 0, fresh = 0, nw = 0, touched = 0;
};

// One candidate block, processed by one wavefront (all 64 lanes).
template <typename S>
__device__ __forceinline__ void fuse_block(const VolumeView &v, const Camera &cam, const FuseCam &fc, uint32_t key,
                                           int lane, FuseAcc &acc)
{
    const int lx = lane & 7, ly = lane >> 3;
    const float2 *__restrict__ pixmap = v.pixmap;
    S *__restrict__ poolT = (S *)v.poolT;
    S *__restrict__ poolP = (S *)v.poolP;
    int bx, by, bz;
    unpack_key(key, bx, by, bz);
    // The decisions run at a raised wave priority, the memory-bound rest of
    // the block at the normal one: a SIMD then issues the arithmetic of the
    // waves that are deciding ahead of the waves that wait on T and P (about
    // 2 % faster than one priority throughout).
    __builtin_amdgcn_s_setprio(2);
    // first probe of the block's hash chain, issued before the decisions so
    // that its latency overlaps them (only this wavefront inserts this key)
    unsigned long long first_entry = 0;
    if (lane == 0) first_entry = v.hash[hash_key(key) & v.hash_mask];
    // x_c = R^T (x - t) = (R00 dx + R10 dy) + R20 dz: the bracket is the
    // lane's (x, y) part, the last term varies with z
    double ax, ay, az;
    {
#pragma clang fp contract(off)
        const double px = v.origin[0] + ((double)(bx * 8 + lx) + 0.5) * v.vs;
        const double py = v.origin[1] + ((double)(by * 8 + ly) + 0.5) * v.vs;
        const double dx = px - cam.t[0];
        const double dy = py - cam.t[1];
        ax = cam.R[0] * dx + cam.R[3] * dy;
        ay = cam.R[1] * dx + cam.R[4] * dy;
        az = cam.R[2] * dx + cam.R[5] * dy;
    }
    // the defined camera coordinates of the column's first voxel (z = 0)
    double x0, y0, z0;
    {
#pragma clang fp contract(off)
        const double pz = v.origin[2] + ((double)(bz * 8) + 0.5) * v.vs;
        const double dz = pz - cam.t[2];
        x0 = ax + cam.R[6] * dz;
        y0 = ay + cam.R[7] * dz;
        z0 = az + cam.R[8] * dz;
    }
    float Tk[8], pk[8];
    uint32_t vmask = 0;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
        // phase 1: approximate camera coordinates and the pixel decision
        int pix[4];
        int exact = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double zf = (double)(4 * half + k);
            const double xc = fma(zf, fc.sx, x0), yc = fma(zf, fc.sy, y0), zc = fma(zf, fc.sz, z0);
            pix[k] = pixel_filter(cam, fc, xc, yc, zc);
            exact |= (pix[k] == -2) << k;
        }
        // phase 2 (rare): voxels the approximation cannot decide take the
        // defined expression
        if (exact) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if ((exact >> k) & 1) {
#pragma clang fp contract(off)
                    const double pz = v.origin[2] + ((double)(bz * 8 + 4 * half + k) + 0.5) * v.vs;
                    const double dz = pz - cam.t[2];
                    const double zc = az + cam.R[8] * dz;
                    pix[k] = zc > 0.0 ? pixel_exact(cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height,
                                                    ax + cam.R[6] * dz, ay + cam.R[7] * dz, zc)
                                      : -1;
                }
            }
        }
        // phase 3: the gathers, issued together (index 0 stands in for misses)
        float2 pm[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) pm[k] = pixmap[pix[k] >= 0 ? pix[k] : 0];
        // phase 4: s = D - z_c, |s| <= delta; the defined z_c where the
        // pixel needed it or s lies near the threshold
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int z = 4 * half + k;
            double sd = (double)pm[k].x - fma((double)z, fc.sz, z0);
            if (((exact >> k) & 1) || fabs(fabs(sd) - v.delta) <= fc.thr_s) {
#pragma clang fp contract(off)
                const double pz = v.origin[2] + ((double)(bz * 8 + z) + 0.5) * v.vs;
                const double dz = pz - cam.t[2];
                sd = (double)pm[k].x - (az + cam.R[8] * dz);
            }
            const bool ok = pix[k] >= 0 && pm[k].x > 0.0f && fabs(sd) <= v.delta;
            Tk[z] = (float)(sd * v.inv_delta);
            pk[z] = pm[k].y;
            vmask |= (uint32_t)ok << z;
        }
    }
    if (lane == 0) {
        uint64_t b = block_linear(v, bx, by, bz);
        atomicAnd(&v.cand_bits[b >> 5], ~(1u << (b & 31)));
    }
    const unsigned long long any = __ballot(vmask != 0);
    if (!any) {
        __builtin_amdgcn_s_setprio(0);
        return;
    }

    int32_t slot = -1;
    int fresh = 0;
    if (lane == 0) {
        const uint32_t k0 = (uint32_t)(first_entry & 0xffffffffu);
        slot = k0 == key ? (int32_t)(first_entry >> 32) : k0 == kEmptyKey ? -1 : hash_find(v, key);
        if (slot < 0) {
            slot = hash_insert_unique(v, key);
            if (slot >= 0) {
                fresh = 1;
                uint64_t b = block_linear(v, bx, by, bz);
                atomicOr(&v.occupancy[b >> 5], 1u << (b & 31));
            }
        }
    }
    slot = __shfl(slot, 0);
    fresh = __shfl(fresh, 0);
    __builtin_amdgcn_s_setprio(0);
    if (slot < 0) return;
    // the block's bound and box as they stand, loaded ahead of the voxel data
    uint32_t old_min = kKeyPosInf, old_box = 0;
    if (lane == 0 && !fresh) {
        old_min = v.block_min[slot];
        old_box = v.block_box[slot];
    }

    S *bt = poolT + (size_t)slot * kBlockVoxels + lane;
    S *bp = poolP + (size_t)slot * kBlockVoxels + lane;
    // lower bound of the block's non-chi values as stored, and the voxels of
    // this lane's column that hold a non-chi value now, both kept for the raycast
    uint32_t kmin = kKeyPosInf, live = 0;
    if (fresh) {
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            const bool m = (vmask >> z) & 1u;
            store_s(bt + 64 * z, m ? Tk[z] : kChi);
            store_s(bp + 64 * z, m ? stored_weight<S>(first_p(v, pk[z])) : 0.0f);
            if (m) kmin = min(kmin, order_key(stored_value<S>(Tk[z])));
        }
        live = vmask;
    } else {
        // phase 5: load every z-slice that holds an update (whole slices:
        // 64 contiguous voxels), then update and store the valid voxels
        uint32_t slices = 0;
#pragma unroll
        for (int z = 0; z < 8; ++z) slices |= (__ballot((vmask >> z) & 1u) != 0ull) << z;
        float T[8], P[8];
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            if ((slices >> z) & 1u) {
                T[z] = load_s(bt + 64 * z);
                P[z] = load_s(bp + 64 * z);
            }
        }
        auto update = [&](auto rule) {
            constexpr int kRule = decltype(rule)::value;
#pragma unroll
            for (int z = 0; z < 8; ++z) {
                if ((vmask >> z) & 1u) {
                    update_voxel<kRule>(v, T[z], P[z], Tk[z], pk[z]);
                    store_s(bt + 64 * z, T[z]);
                    store_s(bp + 64 * z, stored_weight<S>(P[z]));
                    if (fabsf(T[z]) <= 1.0f) {
                        kmin = min(kmin, order_key(stored_value<S>(T[z])));
                        live |= 1u << z;
                    }
                }
            }
        };
        if (v.rule == TSDF_RULE_KALMAN)
            update(std::integral_constant<int, TSDF_RULE_KALMAN>());
        else if (v.rule == TSDF_RULE_RUNNING)
            update(std::integral_constant<int, TSDF_RULE_RUNNING>());
        else
            update(std::integral_constant<int, TSDF_RULE_WEIGHTED>());
    }
    // the owner wavefront folds its new values into the bound (values only
    // ever lower it, so it stays below the true minimum)
    kmin = wave_min_u32(kmin);
    const uint32_t box = wave_box(live);
    if (lane == 0) {
        const uint32_t m = min(old_min, kmin);
        v.block_min[slot] = m;
        v.block_box[slot] = box_union(old_box, box);
        if (v.block_index)
            v.block_index[block_linear(v, bx, by, bz)] = slot | (m > kKeyZero ? kIndexPositive : 0);
    }
    const uint32_t cnt = __popc(vmask);
    acc.upd += cnt;
    acc.fresh += fresh ? cnt : 0u;
    acc.nw += (uint32_t)fresh;   // same value in every lane after the broadcast
    acc.touched += 1u;
}

// Adds a wavefront's counts to the volume's spread counters and clears them.
__device__ __forceinline__ void fuse_flush(const VolumeView &v, FuseAcc &acc, uint32_t wave, int lane)
{
    uint32_t upd = acc.upd, fresh = acc.fresh;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        upd += __shfl_xor(upd, off);
        fresh += __shfl_xor(fresh, off);
    }
    // nw and touched are the same in every lane (wave-uniform updates)
    if (lane == 0 && (upd | acc.nw | acc.touched)) {
        const int l = wave & (kCtrLanes - 1);
        atomicAdd(&v.ctr->frame[l][CTR_UPDATES], (unsigned long long)upd);
        atomicAdd(&v.ctr->total[l][CTR_UPDATES], (unsigned long long)upd);
        atomicAdd(&v.ctr->frame[l][CTR_FRESH], (unsigned long long)fresh);
        atomicAdd(&v.ctr->total[l][CTR_FRESH], (unsigned long long)fresh);
        atomicAdd(&v.ctr->frame[l][CTR_NEW], (unsigned long long)acc.nw);
        atomicAdd(&v.ctr->total[l][CTR_NEW], (unsigned long long)acc.nw);
        atomicAdd(&v.ctr->frame[l][CTR_TOUCHED], (unsigned long long)acc.touched);
        atomicAdd(&v.ctr->total[l][CTR_TOUCHED], (unsigned long long)acc.touched);
    }
    acc = FuseAcc();
}

}  // namespace tsdf

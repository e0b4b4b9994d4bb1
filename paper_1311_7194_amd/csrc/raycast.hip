// Raycast of the block-sparse TSDF into vertex and normal maps (Section 5).
//
// Each ray (through a pixel centre) is sampled at s_n = n * voxel/2, n >= 1.
// A sample's value F is the trilinear interpolation over the 8 voxel
// centres around it; it is invalid if any of them is outside the grid, in
// an unallocated block or chi.  The hit is the first n with both F(s_n) > 0
// and F(s_{n+1}) <= 0 valid; bisection refines it and central differences
// one voxel apart give the normal.
//
// The paper shrinks the traversed range with per-pixel start/end textures
// rasterised from occupied blocks.  Here the march works in voxel-centre
// coordinates q = (x - origin)/voxel - 1/2, where the 8 voxels around a
// sample are floor(q) + {0,1}^3; every sample whose floor(q) lies in an
// unallocated block is provably invalid, so the march jumps over the
// 8-voxel cell of such a block at once using the occupancy bitmap.  Inside
// allocated cells the slots of the cell's block and its 7 upper neighbours
// are cached in registers, so a sample costs 8 loads from the pool.
#include "tsdf_internal.h"

namespace tsdf {

struct Ray {
    double q0[3];   // q at s = 0 (camera centre)
    double dq[3];   // dq/ds
    double o[3];    // world origin
    double d[3];    // unit world direction
};

template <typename S>
__device__ __forceinline__ float ld(const S *p);
template <>
__device__ __forceinline__ float ld<float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float ld<__half>(const __half *p) { return __half2float(*p); }

__device__ __forceinline__ int32_t block_slot(const VolumeView &v, int bx, int by, int bz)
{
    if (bx < 0 || by < 0 || bz < 0 || bx >= v.nblk[0] || by >= v.nblk[1] || bz >= v.nblk[2]) return -1;
    if (!occupied(v, bx, by, bz)) return -1;
    return hash_find(v, pack_key(bx, by, bz));
}

// Cached slots of cell block B and its upper neighbours B + {0,1}^3.
struct SlotCache {
    int B[3];
    int32_t s[8];
};

__device__ __forceinline__ void fill_cache(const VolumeView &v, SlotCache &c, int bx, int by, int bz)
{
    c.B[0] = bx;
    c.B[1] = by;
    c.B[2] = bz;
#pragma unroll
    for (int k = 0; k < 8; ++k) c.s[k] = block_slot(v, bx + (k & 1), by + ((k >> 1) & 1), bz + ((k >> 2) & 1));
}

// Trilinear F at integer base c (global voxel indices) with fractions f,
// using slots from the cache (c must lie in cell c.B).  Returns false when
// invalid.
template <typename S>
__device__ __forceinline__ bool interp_cached(const VolumeView &v, const SlotCache &cache, const int c[3],
                                              const float f[3], float &F)
{
    const S *pool = (const S *)v.poolT;
    const int l0 = c[0] & 7, l1 = c[1] & 7, l2 = c[2] & 7;
    float val[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int ox = k & 1, oy = (k >> 1) & 1, oz = (k >> 2) & 1;
        const int sx = (l0 + ox) >> 3, sy = (l1 + oy) >> 3, sz = (l2 + oz) >> 3;
        const int sel = sx | (sy << 1) | (sz << 2);
        int32_t slot = cache.s[0];
#pragma unroll
        for (int m = 1; m < 8; ++m) slot = (sel == m) ? cache.s[m] : slot;
        if (slot < 0) return false;
        const int vx = (l0 + ox) & 7, vy = (l1 + oy) & 7, vz = (l2 + oz) & 7;
        const float T = ld(pool + (size_t)slot * kBlockVoxels + vx + 8 * vy + 64 * vz);
        if (fabsf(T) > 1.0f) return false;
        val[k] = T;
    }
    const float x00 = val[0] + f[0] * (val[1] - val[0]);
    const float x10 = val[2] + f[0] * (val[3] - val[2]);
    const float x01 = val[4] + f[0] * (val[5] - val[4]);
    const float x11 = val[6] + f[0] * (val[7] - val[6]);
    const float y0 = x00 + f[1] * (x10 - x00);
    const float y1 = x01 + f[1] * (x11 - x01);
    F = y0 + f[2] * (y1 - y0);
    return true;
}

// F at an arbitrary q (uncached lookups; used for refinement and normals).
template <typename S>
__device__ bool interp_at(const VolumeView &v, const double q[3], float &F)
{
    int c[3];
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double fl = floor(q[a]);
        if (!(fl >= 0.0 && fl + 1.0 <= (double)(v.dims[a] - 1))) return false;
        c[a] = (int)fl;
        f[a] = (float)(q[a] - fl);
    }
    SlotCache cache;
    fill_cache(v, cache, c[0] >> 3, c[1] >> 3, c[2] >> 3);
    return interp_cached<S>(v, cache, c, f, F);
}

__device__ __forceinline__ void q_at(const Ray &r, double s, double q[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a] = r.q0[a] + s * r.dq[a];
}

template <typename S>
__global__ __launch_bounds__(256) void raycast_kernel(VolumeView v, Camera cam, float4 *__restrict__ vertex,
                                                      float4 *__restrict__ normal)
{
    // 16x16 pixel tile per workgroup; each wavefront covers 16x4 pixels
    const int i = blockIdx.x * 16 + (threadIdx.x & 15);
    const int j = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= cam.width || j >= cam.height) return;
    const size_t pix = (size_t)j * cam.width + i;
    float4 vout = make_float4(0.f, 0.f, 0.f, 0.f), nout = vout;

    Ray r;
    {
        const double dc0 = (i - cam.cx) / cam.fx, dc1 = (j - cam.cy) / cam.fy;
        const double len = sqrt(dc0 * dc0 + dc1 * dc1 + 1.0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r.d[a] = (cam.R[3 * a] * dc0 + cam.R[3 * a + 1] * dc1 + cam.R[3 * a + 2]) / len;
            r.o[a] = cam.t[a];
            r.q0[a] = (cam.t[a] - v.origin[a]) * v.inv_vs - 0.5;
            r.dq[a] = r.d[a] * v.inv_vs;
        }
    }
    // samples can only be valid while every stencil voxel is inside the grid: q in [0, G-1]
    double s_in = 0.0, s_out = 1e300;
    bool miss = false;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double hiq = (double)(v.dims[a] - 1);
        if (r.dq[a] == 0.0) {
            miss |= (r.q0[a] < 0.0 || r.q0[a] > hiq);
        } else {
            double s0 = (0.0 - r.q0[a]) / r.dq[a], s1 = (hiq - r.q0[a]) / r.dq[a];
            if (s0 > s1) {
                const double tmp = s0;
                s0 = s1;
                s1 = tmp;
            }
            s_in = fmax(s_in, s0);
            s_out = fmin(s_out, s1);
        }
    }
    const double h = 0.5 * v.vs;
    if (!miss && s_in <= s_out) {
        long long n = (long long)ceil(s_in / h) - 1;
        const long long n_end = (long long)floor(s_out / h) + 1;
        if (n < 1) n = 1;
        SlotCache cache;
        cache.B[0] = cache.B[1] = cache.B[2] = -1 << 30;
        bool cell_empty = true;
        float Fprev = 0.0f;
        bool vprev = false;
        long long nprev = -2;
        while (n <= n_end) {
            const double s = (double)n * h;
            double q[3];
            q_at(r, s, q);
            int c[3];
            float f[3];
            bool inside = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double fl = floor(q[a]);
                inside &= (fl >= 0.0 && fl + 1.0 <= (double)(v.dims[a] - 1));
                c[a] = (int)fl;
                f[a] = (float)(q[a] - fl);
            }
            if (!inside) {
                vprev = false;
                ++n;
                continue;
            }
            const int B0 = c[0] >> 3, B1 = c[1] >> 3, B2 = c[2] >> 3;
            if (B0 != cache.B[0] || B1 != cache.B[1] || B2 != cache.B[2]) {
                cache.B[0] = B0;
                cache.B[1] = B1;
                cache.B[2] = B2;
                cell_empty = !occupied(v, B0, B1, B2);
                if (!cell_empty) fill_cache(v, cache, B0, B1, B2);
            }
            if (cell_empty) {
                // jump to the first sample past this cell: every sample before
                // the exit has its base voxel in the empty block
                double s_exit = 1e300;
                const int Bc[3] = {B0, B1, B2};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    if (r.dq[a] > 0.0) s_exit = fmin(s_exit, (8.0 * (Bc[a] + 1) - r.q0[a]) / r.dq[a]);
                    else if (r.dq[a] < 0.0) s_exit = fmin(s_exit, (8.0 * Bc[a] - r.q0[a]) / r.dq[a]);
                }
                long long m = (long long)floor(s_exit / h);
                if (m > n) {
                    // sample m may still sit in the cell; check its base block
                    double qm[3];
                    q_at(r, (double)m * h, qm);
                    const bool still = ((int)floor(qm[0]) >> 3) == B0 && ((int)floor(qm[1]) >> 3) == B1 &&
                                       ((int)floor(qm[2]) >> 3) == B2;
                    n = still ? m + 1 : m;
                } else {
                    n = n + 1;
                }
                vprev = false;
                continue;
            }
            float F;
            const bool valid = interp_cached<S>(v, cache, c, f, F);
            if (valid && vprev && nprev == n - 1 && Fprev > 0.0f && F <= 0.0f) {
                // refine inside [s_{n-1}, s_n]
                double lo = (double)(n - 1) * h, hi = s;
                for (int it = 0; it < 24; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    double qm[3];
                    q_at(r, mid, qm);
                    float Fm;
                    if (!interp_at<S>(v, qm, Fm)) break;
                    if (Fm > 0.0f) lo = mid;
                    else hi = mid;
                }
                const double sh = 0.5 * (lo + hi);
                double qh[3];
                q_at(r, sh, qh);
                float g[3];
                bool ok = true;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    double qp[3] = {qh[0], qh[1], qh[2]}, qn[3] = {qh[0], qh[1], qh[2]};
                    qp[a] += 1.0;
                    qn[a] -= 1.0;
                    float Fp, Fn;
                    ok = ok && interp_at<S>(v, qp, Fp) && interp_at<S>(v, qn, Fn);
                    g[a] = ok ? Fp - Fn : 0.0f;
                }
                const float gl = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
                if (ok && gl > 0.0f) {
                    vout = make_float4((float)(r.o[0] + sh * r.d[0]), (float)(r.o[1] + sh * r.d[1]),
                                       (float)(r.o[2] + sh * r.d[2]), 1.0f);
                    nout = make_float4(g[0] / gl, g[1] / gl, g[2] / gl, 1.0f);
                }
                break;
            }
            Fprev = F;
            vprev = valid;
            nprev = n;
            ++n;
        }
    }
    vertex[pix] = vout;
    normal[pix] = nout;
}

hipError_t launch_raycast(const VolumeView &v, const Camera &cam, float4 *vertex, float4 *normal, hipStream_t s)
{
    dim3 grid((cam.width + 15) / 16, (cam.height + 15) / 16);
    if (v.storage == TSDF_F16)
        hipLaunchKernelGGL(raycast_kernel<__half>, grid, dim3(256), 0, s, v, cam, vertex, normal);
    else
        hipLaunchKernelGGL(raycast_kernel<float>, grid, dim3(256), 0, s, v, cam, vertex, normal);
    return hipGetLastError();
}

}  // namespace tsdf

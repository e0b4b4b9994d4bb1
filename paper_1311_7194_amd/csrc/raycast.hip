// Raycast of the block-sparse TSDF into vertex and normal maps (Section 5).
//
// Each ray (through a pixel centre) is sampled at s_n = n * voxel/2, n >= 1.
// A sample's value F is the trilinear interpolation over the 8 voxel
// centres around it; it is invalid if any of them is outside the grid, in
// an unallocated block or chi.  The hit is the first n with both F(s_n) > 0
// and F(s_{n+1}) <= 0 valid; bisection refines it and central differences
// one voxel apart give the normal.
//
// Range shrinking.  The paper rasterises the faces of occupied blocks into
// per-pixel start and end textures so that rays only traverse the depth span
// of occupied blocks.  Here a compute pass does the same per 8x8 pixel tile:
// for every allocated block it projects the box in which that block is the
// base of the interpolation stencil and widens the [min, max] camera depth of
// every tile the box covers.  Every valid sample lies in such a box, so
// starting and ending each ray at its tile's span skips only invalid samples.
//
// Empty-space skipping inside the span.  The march works in voxel-centre
// coordinates q = (x - origin)/voxel - 1/2, where the 8 voxels around a
// sample are floor(q) + {0,1}^3; a sample whose floor(q) lies in an
// unallocated block is provably invalid, so the march jumps over the 8-voxel
// cell of such a block at once (occupancy bitmap).  Inside allocated cells
// the slots of the cell's block and its 7 upper neighbours stay in registers.
#include "tsdf_internal.h"

namespace tsdf {

constexpr int kRT = 8;                      // raycast tile edge in pixels
constexpr uint32_t kInfBits = 0x7f800000u;  // +inf as float bits

// ------------------------------------------------------------ range pass

__global__ __launch_bounds__(256) void range_kernel(VolumeView v, Camera cam, uint32_t stamp, int tiles_x,
                                                    int tiles_y)
{
    const uint32_t n = min(v.state->pool_count, v.capacity);
    uint32_t *tmin = v.tile_range;
    uint32_t *tmax = v.tile_range + (size_t)tiles_x * tiles_y;
    // camera axes in float: x_c = R^T (x - t)
    const float R[9] = {(float)cam.R[0], (float)cam.R[1], (float)cam.R[2], (float)cam.R[3], (float)cam.R[4],
                        (float)cam.R[5], (float)cam.R[6], (float)cam.R[7], (float)cam.R[8]};
    const float fx = (float)cam.fx, fy = (float)cam.fy, cx = (float)cam.cx, cy = (float)cam.cy;
    const float bw = (float)(8.0 * v.vs);
    for (uint32_t slot = blockIdx.x * 256u + threadIdx.x; slot < n; slot += gridDim.x * 256u) {
        int bx, by, bz;
        unpack_key(v.pool_keys[slot], bx, by, bz);
        // stencil-base box of block B: q in [8B, 8B + 8], x = origin + (q + 1/2) voxel;
        // its min corner relative to the camera centre, in double then float
        const float ox = (float)(v.origin[0] + (8.0 * bx + 0.5) * v.vs - cam.t[0]);
        const float oy = (float)(v.origin[1] + (8.0 * by + 0.5) * v.vs - cam.t[1]);
        const float oz = (float)(v.origin[2] + (8.0 * bz + 0.5) * v.vs - cam.t[2]);
        float zlo = 3.4e38f, zhi = -3.4e38f, ulo = 3.4e38f, uhi = -3.4e38f, vlo = 3.4e38f, vhi = -3.4e38f;
        bool behind = false;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float dx = ox + ((k & 1) ? bw : 0.0f), dy = oy + ((k & 2) ? bw : 0.0f),
                        dz = oz + ((k & 4) ? bw : 0.0f);
            const float xc = R[0] * dx + R[3] * dy + R[6] * dz;
            const float yc = R[1] * dx + R[4] * dy + R[7] * dz;
            const float zc = R[2] * dx + R[5] * dy + R[8] * dz;
            zlo = fminf(zlo, zc);
            zhi = fmaxf(zhi, zc);
            behind |= !(zc > 1e-4f);
            const float rz = 1.0f / zc;
            ulo = fminf(ulo, fx * xc * rz + cx);
            uhi = fmaxf(uhi, fx * xc * rz + cx);
            vlo = fminf(vlo, fy * yc * rz + cy);
            vhi = fmaxf(vhi, fy * yc * rz + cy);
        }
        if (zhi <= 0.0f) continue;            // wholly behind the camera
        if (behind) {                         // reaches the camera plane: rays start at the camera
            v.state->near_stamp = stamp;
            continue;
        }
        // pixel centres (i, j) inside the projected box, widened by a pixel
        const int i0 = max((int)floorf(ulo) - 1, 0), i1 = min((int)ceilf(uhi) + 1, cam.width - 1);
        const int j0 = max((int)floorf(vlo) - 1, 0), j1 = min((int)ceilf(vhi) + 1, cam.height - 1);
        if (i0 > i1 || j0 > j1) continue;
        const uint32_t zl = __float_as_uint(fmaxf(zlo * (1.0f - 1e-5f) - 1e-6f, 0.0f));
        const uint32_t zh = __float_as_uint(zhi * (1.0f + 1e-5f) + 1e-6f);
        for (int tj = j0 / kRT; tj <= j1 / kRT; ++tj)
            for (int ti = i0 / kRT; ti <= i1 / kRT; ++ti) {
                const size_t t = (size_t)tj * tiles_x + ti;
                if (tmin[t] > zl) atomicMin(&tmin[t], zl);
                if (tmax[t] < zh) atomicMax(&tmax[t], zh);
            }
    }
}

// ------------------------------------------------------------ march

struct Ray {
    double q0[3];    // q at s = 0 (camera centre)
    double dq[3];    // dq/ds
    double inv[3];   // ds/dq (0 where the ray is parallel to the axis)
    double d[3];     // unit world direction
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
// using slots from the cache (c must lie in cell c.B).  False when invalid.
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

// F at an arbitrary q, refilling the slot cache only when the stencil's
// base block changes (refinement and normals).
template <typename S>
__device__ __forceinline__ bool interp_q(const VolumeView &v, SlotCache &cache, const double q[3], float &F)
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
    if ((c[0] >> 3) != cache.B[0] || (c[1] >> 3) != cache.B[1] || (c[2] >> 3) != cache.B[2])
        fill_cache(v, cache, c[0] >> 3, c[1] >> 3, c[2] >> 3);
    return interp_cached<S>(v, cache, c, f, F);
}

__device__ __forceinline__ void q_at(const Ray &r, double s, double q[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a] = r.q0[a] + s * r.dq[a];
}

template <typename S>
__global__ __launch_bounds__(256) void raycast_kernel(VolumeView v, Camera cam, uint32_t stamp, int tiles_x,
                                                      int tiles_y, float4 *__restrict__ vertex,
                                                      float4 *__restrict__ normal)
{
    // one wavefront per 8x8 pixel tile, 2x2 tiles per workgroup
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ti = blockIdx.x * 2 + (w & 1), tj = blockIdx.y * 2 + (w >> 1);
    if (ti >= tiles_x || tj >= tiles_y) return;
    const size_t t = (size_t)tj * tiles_x + ti;
    uint32_t *tmin = v.tile_range;
    uint32_t *tmax = v.tile_range + (size_t)tiles_x * tiles_y;
    const uint32_t zmin_bits = tmin[t], zmax_bits = tmax[t];
    const float zmin_t = __uint_as_float(zmin_bits);
    const float zmax_t = __uint_as_float(zmax_bits);
    const bool near = v.state->near_stamp == stamp;
    // this wavefront is the tile's only reader: clear it for the next raycast
    // (the stores depend on the loaded values, so they follow the loads)
    if (lane == 0) {
        if (zmin_bits != kInfBits) tmin[t] = kInfBits;
        if (zmax_bits != 0u) tmax[t] = 0u;
    }
    const int i = ti * kRT + (lane & 7), j = tj * kRT + (lane >> 3);
    if (i >= cam.width || j >= cam.height) return;
    const size_t pix = (size_t)j * cam.width + i;
    float4 vout = make_float4(0.f, 0.f, 0.f, 0.f), nout = vout;

    // march: find the first front-facing bracket [s_lo, s_hi]
    Ray r;
    SlotCache cache;
    cache.B[0] = cache.B[1] = cache.B[2] = -(1 << 30);
    bool hit = false;
    double s_lo = 0.0, s_hi = 0.0;
    float F_lo = 0.0f, F_hi = 0.0f;
    if (near || zmin_t <= zmax_t) {
        const double dc0 = (i - cam.cx) / cam.fx, dc1 = (j - cam.cy) / cam.fy;
        const double len = sqrt(dc0 * dc0 + dc1 * dc1 + 1.0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            r.d[a] = (cam.R[3 * a] * dc0 + cam.R[3 * a + 1] * dc1 + cam.R[3 * a + 2]) / len;
            r.q0[a] = (cam.t[a] - v.origin[a]) * v.inv_vs - 0.5;
            r.dq[a] = r.d[a] * v.inv_vs;
            r.inv[a] = r.dq[a] != 0.0 ? 1.0 / r.dq[a] : 0.0;
        }
        // valid samples need every stencil voxel in the grid: q in [0, G-1]
        double s_in = 0.0, s_out = 1e300;
        bool miss = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double hiq = (double)(v.dims[a] - 1);
            if (r.dq[a] == 0.0) {
                miss |= (r.q0[a] < 0.0 || r.q0[a] > hiq);
            } else {
                const double s0 = (0.0 - r.q0[a]) * r.inv[a], s1 = (hiq - r.q0[a]) * r.inv[a];
                s_in = fmax(s_in, fmin(s0, s1));
                s_out = fmin(s_out, fmax(s0, s1));
            }
        }
        // the tile's depth span (camera z = s / len along this ray)
        if (!near) {
            s_in = fmax(s_in, (double)zmin_t * len);
            s_out = fmin(s_out, (double)zmax_t * len);
        }
        const double h = 0.5 * v.vs;
        if (!miss && s_in <= s_out) {
            long long n = (long long)floor(s_in / h) - 1;
            const long long n_end = (long long)ceil(s_out / h) + 1;
            if (n < 1) n = 1;
            bool cell_empty = true;
            float Fprev = 0.0f;
            bool vprev = false;
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
                    c[a] = inside ? (int)fl : 0;
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
                    if (!cell_empty) {
                        fill_cache(v, cache, B0, B1, B2);
                    } else {
#pragma unroll
                        for (int k = 0; k < 8; ++k) cache.s[k] = -1;   // keeps the cache consistent with B
                    }
                }
                if (cell_empty) {
                    // jump to the first sample past this cell: every sample
                    // before the exit has its base voxel in the empty block
                    double s_exit = 1e300;
                    const int Bc[3] = {B0, B1, B2};
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        if (r.dq[a] > 0.0) s_exit = fmin(s_exit, (8.0 * (Bc[a] + 1) - r.q0[a]) * r.inv[a]);
                        else if (r.dq[a] < 0.0) s_exit = fmin(s_exit, (8.0 * Bc[a] - r.q0[a]) * r.inv[a]);
                    }
                    const long long m = (long long)floor(s_exit / h);
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
                if (valid && vprev && Fprev > 0.0f && F <= 0.0f) {
                    hit = true;
                    s_lo = (double)(n - 1) * h;
                    s_hi = s;
                    F_lo = Fprev;
                    F_hi = F;
                    break;
                }
                Fprev = F;
                vprev = valid;
                ++n;
            }
        }
    }
    // refinement with every lane converged: 12 bisection steps inside the
    // bracket (F > 0 at s_lo, F <= 0 at s_hi) leave it 1/8192 voxel wide; a
    // linear interpolation inside it gives the root, then central differences
    if (hit) {
        double a = s_lo, b = s_hi;
        float Fa = F_lo, Fb = F_hi;
        for (int it = 0; it < 12; ++it) {
            const double mid = 0.5 * (a + b);
            double qm[3];
            q_at(r, mid, qm);
            float Fm;
            if (!interp_q<S>(v, cache, qm, Fm)) break;
            if (Fm > 0.0f) {
                a = mid;
                Fa = Fm;
            } else {
                b = mid;
                Fb = Fm;
            }
        }
        const double sm = (Fa - Fb) > 0.0f ? a + (b - a) * ((double)Fa / ((double)Fa - (double)Fb)) : 0.5 * (a + b);
        double qh[3];
        q_at(r, sm, qh);
        float g[3];
        bool ok = true;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            double qp[3] = {qh[0], qh[1], qh[2]}, qn[3] = {qh[0], qh[1], qh[2]};
            qp[ax] += 1.0;
            qn[ax] -= 1.0;
            float Fp = 0.0f, Fn = 0.0f;
            ok = ok && interp_q<S>(v, cache, qp, Fp) && interp_q<S>(v, cache, qn, Fn);
            g[ax] = Fp - Fn;
        }
        const float gl = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        if (ok && gl > 0.0f) {
            vout = make_float4((float)(cam.t[0] + sm * r.d[0]), (float)(cam.t[1] + sm * r.d[1]),
                               (float)(cam.t[2] + sm * r.d[2]), 1.0f);
            nout = make_float4(g[0] / gl, g[1] / gl, g[2] / gl, 1.0f);
        }
    }
    vertex[pix] = vout;
    normal[pix] = nout;
}

hipError_t launch_raycast(const VolumeView &v, const Camera &cam, uint32_t stamp, float4 *vertex, float4 *normal,
                          hipStream_t s)
{
    const int tiles_x = (cam.width + kRT - 1) / kRT, tiles_y = (cam.height + kRT - 1) / kRT;
    // range pass over the allocated blocks (grid-stride; the block count stays on the device)
    hipLaunchKernelGGL(range_kernel, dim3(2048), dim3(256), 0, s, v, cam, stamp, tiles_x, tiles_y);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid((tiles_x + 1) / 2, (tiles_y + 1) / 2);
    if (v.storage == TSDF_F16)
        hipLaunchKernelGGL(raycast_kernel<__half>, grid, dim3(256), 0, s, v, cam, stamp, tiles_x, tiles_y, vertex,
                           normal);
    else
        hipLaunchKernelGGL(raycast_kernel<float>, grid, dim3(256), 0, s, v, cam, stamp, tiles_x, tiles_y, vertex,
                           normal);
    return hipGetLastError();
}

}  // namespace tsdf

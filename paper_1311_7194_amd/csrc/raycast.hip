// Raycast of the block-sparse TSDF into vertex and normal maps (Section 5).
//
// Each ray (through a pixel centre) is sampled at s_n = n * voxel/2, n >= 1.
// A sample's value F is the trilinear interpolation over the 8 voxel
// centres around it; it is invalid if any of them is outside the grid, in
// an unallocated block or chi.  The hit is the first n with both F(s_n) > 0
// and F(s_{n+1}) <= 0 valid; the bracket is refined to the root and central
// differences one voxel apart give the normal.
//
// Range shrinking.  The paper rasterises the faces of occupied blocks into
// per-pixel start and end textures so that rays only traverse the depth span
// of occupied blocks.  Here a compute pass does the same per 8x8 pixel tile:
// for every allocated block it projects the box in which that block is the
// base of the interpolation stencil and widens the [min, max] camera depth of
// every tile the box covers.  Every valid sample lies in such a box, so
// starting and ending each ray at its tile's span skips only invalid samples.
//
// March.  A group of G lanes marches one ray: lane j evaluates sample
// n_base + j, shuffles pair every sample with its predecessor and a ballot
// finds the first crossing, so a ray advances G samples per step.  Samples
// live in voxel-centre coordinates q = (x - origin)/voxel - 1/2, where the 8
// voxels around a sample are floor(q) + {0,1}^3.  When the group's last
// sample lies in a cell whose base block is unallocated, every sample up to
// the cell's exit is invalid and the group jumps past it; when all 8 blocks
// that the cell's stencils reach hold only positive values, no crossing can
// end inside the cell and the group jumps to the cell's last sample.
#include "tsdf_internal.h"

namespace tsdf {

constexpr int kRT = 8;                      // raycast tile edge in pixels
constexpr uint32_t kInfBits = 0x7f800000u;  // +inf as float bits

// ------------------------------------------------------------ range pass

__global__ void range_clear_kernel(uint32_t *tile_range, int n_tiles)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n_tiles) {
        tile_range[t] = kInfBits;
        tile_range[n_tiles + t] = 0u;
    }
}

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

// Cached slots of cell block B and its upper neighbours B + {0,1}^3, and
// whether every non-chi value in those 8 blocks is positive (then no sample
// of the cell can have F <= 0: F is a convex combination of them).
struct SlotCache {
    int B[3];
    int32_t s[8];
    bool positive;
};

// Dense index: one load per neighbour; the entry carries the block's sign flag.
template <bool kDense>
__device__ __forceinline__ void fill_cache(const VolumeView &v, SlotCache &c, int bx, int by, int bz)
{
    c.B[0] = bx;
    c.B[1] = by;
    c.B[2] = bz;
    bool pos = true;
    if constexpr (kDense) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int x = bx + (k & 1), y = by + ((k >> 1) & 1), z = bz + ((k >> 2) & 1);
            const bool in = x < v.nblk[0] && y < v.nblk[1] && z < v.nblk[2];
            const int32_t e = in ? v.block_index[block_linear(v, x, y, z)] : -1;
            c.s[k] = e < 0 ? -1 : (e & kIndexSlotMask);
            pos &= (e < 0) || (e & kIndexPositive);
        }
    } else {
        uint32_t kmin = kKeyPosInf;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int x = bx + (k & 1), y = by + ((k >> 1) & 1), z = bz + ((k >> 2) & 1);
            int32_t sl = -1;
            if (x < v.nblk[0] && y < v.nblk[1] && z < v.nblk[2] && occupied(v, x, y, z))
                sl = hash_find(v, pack_key(x, y, z));
            c.s[k] = sl;
            if (sl >= 0) kmin = min(kmin, v.block_min[sl]);
        }
        pos = kmin > kKeyZero;
    }
    c.positive = pos;
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
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int ox = k & 1, oy = (k >> 1) & 1, oz = (k >> 2) & 1;
        const int sx = (l0 + ox) >> 3, sy = (l1 + oy) >> 3, sz = (l2 + oz) >> 3;
        const int sel = sx | (sy << 1) | (sz << 2);
        int32_t slot = cache.s[0];
#pragma unroll
        for (int m = 1; m < 8; ++m) slot = (sel == m) ? cache.s[m] : slot;
        const int vx = (l0 + ox) & 7, vy = (l1 + oy) & 7, vz = (l2 + oz) & 7;
        const float T = slot >= 0 ? ld(pool + (size_t)slot * kBlockVoxels + vx + 8 * vy + 64 * vz) : kChi;
        ok &= fabsf(T) <= 1.0f;
        val[k] = T;
    }
    const float x00 = val[0] + f[0] * (val[1] - val[0]);
    const float x10 = val[2] + f[0] * (val[3] - val[2]);
    const float x01 = val[4] + f[0] * (val[5] - val[4]);
    const float x11 = val[6] + f[0] * (val[7] - val[6]);
    const float y0 = x00 + f[1] * (x10 - x00);
    const float y1 = x01 + f[1] * (x11 - x01);
    F = y0 + f[2] * (y1 - y0);
    return ok;
}

__device__ __forceinline__ void q_at(const Ray &r, double s, double q[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) q[a] = r.q0[a] + s * r.dq[a];
}

// Stencil base voxel and fractions of q; false outside the grid.
__device__ __forceinline__ bool stencil(const VolumeView &v, const double q[3], int c[3], float f[3])
{
    bool inside = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double fl = floor(q[a]);
        inside &= (fl >= 0.0 && fl + 1.0 <= (double)(v.dims[a] - 1));
        c[a] = inside ? (int)fl : 0;
        f[a] = (float)(q[a] - fl);
    }
    return inside;
}

// F at q, refilling the lane's cache when the stencil's base block changes.
template <typename S, bool kDense>
__device__ __forceinline__ bool sample_q(const VolumeView &v, SlotCache &cache, const double q[3], float &F)
{
    int c[3];
    float f[3];
    if (!stencil(v, q, c, f)) return false;
    if ((c[0] >> 3) != cache.B[0] || (c[1] >> 3) != cache.B[1] || (c[2] >> 3) != cache.B[2])
        fill_cache<kDense>(v, cache, c[0] >> 3, c[1] >> 3, c[2] >> 3);
    return interp_cached<S>(v, cache, c, f, F);
}

// First lattice index past the cell of block B along the ray (the caller's
// samples before it all have their base voxel in B).
__device__ __forceinline__ long long cell_exit_sample(const Ray &r, const int B[3], double h)
{
    double s_exit = 1e300;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (r.dq[a] > 0.0) s_exit = fmin(s_exit, (8.0 * (B[a] + 1) - r.q0[a]) * r.inv[a]);
        else if (r.dq[a] < 0.0) s_exit = fmin(s_exit, (8.0 * B[a] - r.q0[a]) * r.inv[a]);
    }
    const long long m = (long long)floor(s_exit / h);
    double qm[3];
    q_at(r, (double)m * h, qm);
    const bool still = ((int)floor(qm[0]) >> 3) == B[0] && ((int)floor(qm[1]) >> 3) == B[1] &&
                       ((int)floor(qm[2]) >> 3) == B[2];
    return still ? m + 1 : m;
}

// Shuffle inside a group of G lanes: value of lane `src` of this lane's group.
template <int G>
__device__ __forceinline__ int group_lane(int lane, int src) { return (lane & ~(G - 1)) | src; }

template <typename S, int G, bool kDense>
__global__ __launch_bounds__(256) void raycast_kernel(VolumeView v, Camera cam, uint32_t stamp, int tiles_x,
                                                      int tiles_y, float4 *__restrict__ vertex,
                                                      float4 *__restrict__ normal)
{
    static_assert(G >= 1 && G <= 16 && (G & (G - 1)) == 0, "group size");
    const int lane = threadIdx.x & 63;
    const int j = lane & (G - 1);                       // sample slot inside the ray's group
    // rays in 8x8-pixel tile order: 64 consecutive rays form one tile
    const long long ray = ((long long)blockIdx.x * 256 + threadIdx.x) / G;
    const long long tile = ray >> 6;
    const int within = (int)(ray & 63);
    const int ti = (int)(tile % tiles_x), tj = (int)(tile / tiles_x);
    const int i = ti * kRT + (within & 7), jpix = tj * kRT + (within >> 3);
    const bool active = tj < tiles_y && i < cam.width && jpix < cam.height;
    const double h = 0.5 * v.vs;

    Ray r;
    long long n_lo = 1, n_end = 0;
    if (active) {
        const size_t t = (size_t)tj * tiles_x + ti;
        const float zmin_t = __uint_as_float(v.tile_range[t]);
        const float zmax_t = __uint_as_float(v.tile_range[(size_t)tiles_x * tiles_y + t]);
        const bool near = v.state->near_stamp == stamp;
        const double dc0 = (i - cam.cx) / cam.fx, dc1 = (jpix - cam.cy) / cam.fy;
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
        bool miss = !(near || zmin_t <= zmax_t);
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
        if (!near) {   // the tile's depth span (camera z = s / len along this ray)
            s_in = fmax(s_in, (double)zmin_t * len);
            s_out = fmin(s_out, (double)zmax_t * len);
        }
        if (!miss && s_in <= s_out) {
            n_lo = max((long long)floor(s_in / h) - 1, 1ll);
            n_end = (long long)ceil(s_out / h) + 1;
        }
    }

    // ---- march: the group evaluates samples n_base .. n_base + G - 1 per step
    SlotCache cache;
    cache.B[0] = cache.B[1] = cache.B[2] = -(1 << 30);
    long long n_base = n_lo;
    bool done = !(active && n_lo <= n_end);
    bool hit = false;
    float Fc = 0.0f;     // carried last sample of the previous step (valid flag vc)
    bool vc = false;
    double s_lo = 0.0, s_hi = 0.0;
    float F_lo = 0.0f, F_hi = 0.0f;
    while (__ballot(!done)) {
        const long long n = n_base + j;
        bool valid = false, cell_empty = false, in_cell = false;
        float F = 0.0f;
        if (!done && n <= n_end) {
            double q[3];
            q_at(r, (double)n * h, q);
            int c[3];
            float f[3];
            if (stencil(v, q, c, f)) {
                if ((c[0] >> 3) != cache.B[0] || (c[1] >> 3) != cache.B[1] || (c[2] >> 3) != cache.B[2])
                    fill_cache<kDense>(v, cache, c[0] >> 3, c[1] >> 3, c[2] >> 3);
                in_cell = true;   // the cache now describes this sample's cell
                cell_empty = cache.s[0] < 0;
                if (!cell_empty) valid = interp_cached<S>(v, cache, c, f, F);
            }
        }
        // pair every sample with its predecessor (lane j - 1, or the carry)
        const float Fp_sh = __shfl(F, group_lane<G>(lane, (j + G - 1) & (G - 1)));
        const bool vp_sh = __shfl((int)valid, group_lane<G>(lane, (j + G - 1) & (G - 1))) != 0;
        const float Fp = j == 0 ? Fc : Fp_sh;
        const bool vp = j == 0 ? vc : vp_sh;
        const bool cross = !done && n <= n_end && valid && vp && Fp > 0.0f && F <= 0.0f;
        const unsigned long long m = __ballot(cross);
        const uint32_t gm = (uint32_t)(m >> (lane & ~(G - 1))) & ((G == 32 ? 0xffffffffu : (1u << G) - 1u));
        // (done and gm are the same in every lane of a group, so the group's
        // lanes all take part in these shuffles)
        if (!done && gm) {
            const int first = __builtin_ctz(gm);
            const long long nh = n_base + first;
            s_lo = (double)(nh - 1) * h;
            s_hi = (double)nh * h;
            F_lo = __shfl(Fp, group_lane<G>(lane, first));
            F_hi = __shfl(F, group_lane<G>(lane, first));
            hit = true;
            done = true;
        }
        // advance: the group's last lane decides a jump over its cell
        const int last = G - 1;
        const float F_last = __shfl(F, group_lane<G>(lane, last));
        const bool v_last = __shfl((int)valid, group_lane<G>(lane, last)) != 0;
        const bool empty_last = __shfl((int)(in_cell && cell_empty), group_lane<G>(lane, last)) != 0;
        const bool pos_last = __shfl((int)(in_cell && !cell_empty && cache.positive), group_lane<G>(lane, last)) != 0;
        const int B0 = __shfl(cache.B[0], group_lane<G>(lane, last));
        const int B1 = __shfl(cache.B[1], group_lane<G>(lane, last));
        const int B2 = __shfl(cache.B[2], group_lane<G>(lane, last));
        if (!done) {
            const long long n_last = n_base + last;
            long long next = n_last + 1;
            bool carry = true;
            if (n_last > n_end) {
                done = true;
            } else if (empty_last || pos_last) {
                const int Bc[3] = {B0, B1, B2};
                const long long exit_n = cell_exit_sample(r, Bc, h);   // first sample past the cell
                // empty: every sample before the exit is invalid; positive: none
                // before the cell's last sample can end a crossing
                const long long target = empty_last ? exit_n : exit_n - 1;
                if (target > next) {
                    next = target;
                    carry = false;
                }
            }
            Fc = carry ? F_last : 0.0f;
            vc = carry && v_last;
            n_base = next;
            if (n_base > n_end) done = true;
        }
    }

    // ---- refinement: G-ary search inside [s_lo, s_hi] (F_lo > 0 >= F_hi)
    constexpr int kSteps = G == 1 ? 13 : G == 2 ? 9 : G == 4 ? 6 : G == 8 ? 5 : 4;
    double a = s_lo, b = s_hi;
    float Fa = F_lo, Fb = F_hi;
    bool refine = hit;
    for (int it = 0; it < kSteps; ++it) {
        if (!__ballot(refine)) break;
        float Fm = 0.0f;
        bool vm = false;
        const double sm = a + (b - a) * (double)(j + 1) / (double)(G + 1);
        if (refine) {
            double qm[3];
            q_at(r, sm, qm);
            vm = sample_q<S, kDense>(v, cache, qm, Fm);
        }
        const uint32_t bad = (uint32_t)(__ballot(refine && !vm) >> (lane & ~(G - 1))) & ((1u << G) - 1u);
        const uint32_t neg = (uint32_t)(__ballot(refine && vm && Fm <= 0.0f) >> (lane & ~(G - 1))) & ((1u << G) - 1u);
        // first non-positive point k: the root lies in (point k-1, point k];
        // refine is the same in every lane of a group
        const int k = neg ? __builtin_ctz(neg) : G;
        const float F_km1 = __shfl(Fm, group_lane<G>(lane, (k + G - 1) & (G - 1)));
        const float F_k = __shfl(Fm, group_lane<G>(lane, k & (G - 1)));
        if (refine) {
            if (bad) {
                refine = false;   // an invalid point inside the bracket: keep the bracket
            } else {
                const double na = k == 0 ? a : a + (b - a) * (double)k / (double)(G + 1);
                const double nb = k == G ? b : a + (b - a) * (double)(k + 1) / (double)(G + 1);
                Fa = k == 0 ? Fa : F_km1;
                Fb = k == G ? Fb : F_k;
                a = na;
                b = nb;
            }
        }
    }
    const double sh = hit ? ((Fa - Fb) > 0.0f ? a + (b - a) * ((double)Fa / ((double)Fa - (double)Fb)) : 0.5 * (a + b))
                          : 0.0;
    // ---- normal: central differences one voxel apart, lanes share the 6 samples
    float g[3] = {0.f, 0.f, 0.f};
    bool ok = hit;
    if (__ballot(hit)) {
        double qh[3];
        q_at(r, sh, qh);
        float Fs[6];
        bool vs[6];
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            Fs[e] = 0.0f;
            vs[e] = false;
        }
        // sample e in {+x, -x, +y, -y, +z, -z} is taken by lane e % G of the group
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            if (hit && (e % G) == j) {
                double qe[3] = {qh[0], qh[1], qh[2]};
                qe[e >> 1] += (e & 1) ? -1.0 : 1.0;
                vs[e] = sample_q<S, kDense>(v, cache, qe, Fs[e]);
            }
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const int src = group_lane<G>(lane, e % G);
            Fs[e] = __shfl(Fs[e], src);
            vs[e] = __shfl((int)vs[e], src) != 0;
            ok = ok && vs[e];
        }
        g[0] = Fs[0] - Fs[1];
        g[1] = Fs[2] - Fs[3];
        g[2] = Fs[4] - Fs[5];
    }
    if (active && j == 0) {
        float4 vout = make_float4(0.f, 0.f, 0.f, 0.f), nout = vout;
        const float gl = sqrtf(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        if (ok && gl > 0.0f) {
            vout = make_float4((float)(cam.t[0] + sh * r.d[0]), (float)(cam.t[1] + sh * r.d[1]),
                               (float)(cam.t[2] + sh * r.d[2]), 1.0f);
            nout = make_float4(g[0] / gl, g[1] / gl, g[2] / gl, 1.0f);
        }
        const size_t pix = (size_t)jpix * cam.width + i;
        vertex[pix] = vout;
        normal[pix] = nout;
    }
}

template <typename S, bool kDense>
static void launch_group(int G, dim3 grid, hipStream_t s, const VolumeView &v, const Camera &cam, uint32_t stamp,
                         int tx, int ty, float4 *vertex, float4 *normal)
{
    switch (G) {
    case 1: hipLaunchKernelGGL((raycast_kernel<S, 1, kDense>), grid, dim3(256), 0, s, v, cam, stamp, tx, ty, vertex, normal); break;
    case 2: hipLaunchKernelGGL((raycast_kernel<S, 2, kDense>), grid, dim3(256), 0, s, v, cam, stamp, tx, ty, vertex, normal); break;
    case 4: hipLaunchKernelGGL((raycast_kernel<S, 4, kDense>), grid, dim3(256), 0, s, v, cam, stamp, tx, ty, vertex, normal); break;
    case 16: hipLaunchKernelGGL((raycast_kernel<S, 16, kDense>), grid, dim3(256), 0, s, v, cam, stamp, tx, ty, vertex, normal); break;
    default: hipLaunchKernelGGL((raycast_kernel<S, 8, kDense>), grid, dim3(256), 0, s, v, cam, stamp, tx, ty, vertex, normal); break;
    }
}

hipError_t launch_raycast(const VolumeView &v, const Camera &cam, uint32_t stamp, int group, float4 *vertex,
                          float4 *normal, hipStream_t s)
{
    const int tiles_x = (cam.width + kRT - 1) / kRT, tiles_y = (cam.height + kRT - 1) / kRT;
    const int n_tiles = tiles_x * tiles_y;
    hipLaunchKernelGGL(range_clear_kernel, dim3((n_tiles + 255) / 256), dim3(256), 0, s, v.tile_range, n_tiles);
    // range pass over the allocated blocks (grid-stride; the block count stays on the device)
    hipLaunchKernelGGL(range_kernel, dim3(2048), dim3(256), 0, s, v, cam, stamp, tiles_x, tiles_y);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int G = (group == 1 || group == 2 || group == 4 || group == 16) ? group : 8;
    const long long threads = (long long)n_tiles * 64 * G;
    dim3 grid((unsigned)((threads + 255) / 256));
    const bool dense = v.block_index != nullptr;
    if (v.storage == TSDF_F16) {
        if (dense) launch_group<__half, true>(G, grid, s, v, cam, stamp, tiles_x, tiles_y, vertex, normal);
        else launch_group<__half, false>(G, grid, s, v, cam, stamp, tiles_x, tiles_y, vertex, normal);
    } else {
        if (dense) launch_group<float, true>(G, grid, s, v, cam, stamp, tiles_x, tiles_y, vertex, normal);
        else launch_group<float, false>(G, grid, s, v, cam, stamp, tiles_x, tiles_y, vertex, normal);
    }
    return hipGetLastError();
}

}  // namespace tsdf

// Device bodies of the range pass and the raycast march, shared by the
// single-volume kernels (raycast.hip) and the batched kernels (batch.hip).
// See raycast.hip for the method.
#pragma once

#include "tsdf_internal.h"

namespace tsdf {

constexpr int kRT = 8;                      // raycast tile edge in pixels
constexpr uint32_t kInfBits = 0x7f800000u;  // +inf as float bits
constexpr int kCellFootprint = 64;          // largest footprint (cells) a block widens cell by cell
constexpr uint32_t kInfoEmpty = 1u << 30;    // march: the sample's cell block is absent
constexpr uint32_t kInfoPositive = 1u << 31; // march: every value the cell's stencils reach is positive

// ------------------------------------------------------------ range maps

constexpr int kCellsPerTile = kRT / kCell;   // cells along a tile edge

// Clears the depth spans of one frame: thread gt of a launch space of
// (tiles x 64) clears cell `gt % 64` of tile `gt / 64` (if the tile has that
// many cells), and the tile itself.
__device__ __forceinline__ void range_clear_body(const VolumeView &v, int tiles_x, int tiles_y, int width,
                                                 int height, long long gt)
{
    const long long tile = gt >> 6;
    const int within = (int)(gt & 63);
    const long long nt = (long long)tiles_x * tiles_y;
    if (tile >= nt) return;
    if (within == 0) {
        v.tile_range[tile] = kInfBits;
        v.tile_range[nt + tile] = 0u;
    }
    if (within >= kCellsPerTile * kCellsPerTile) return;
    const int cw = (width + kCell - 1) / kCell, ch = (height + kCell - 1) / kCell;
    const int ci = (int)(tile % tiles_x) * kCellsPerTile + within % kCellsPerTile;
    const int cj = (int)(tile / tiles_x) * kCellsPerTile + within / kCellsPerTile;
    if (ci < cw && cj < ch) {
        const size_t c = (size_t)cj * cw + ci;
        v.pix_range[c] = kInfBits;
        v.pix_range[(size_t)cw * ch + c] = 0u;
    }
}

// ------------------------------------------------------------ range pass

// Cell spans gathered in LDS by one workgroup before they go to memory:
// consecutive pool slots are neighbours in space, so their blocks widen the
// same cells, and one pair of memory atomics per distinct cell replaces one
// per block.  Keys are (scene << 26) | cell.
constexpr int kSpanLds = 2048;
constexpr uint32_t kSpanEmpty = 0xffffffffu;
struct SpanLds {
    uint32_t key[kSpanLds], lo[kSpanLds], hi[kSpanLds];
};

__device__ __forceinline__ void span_lds_init(SpanLds &L)
{
    for (int e = threadIdx.x; e < kSpanLds; e += blockDim.x) {
        L.key[e] = kSpanEmpty;
        L.lo[e] = kInfBits;
        L.hi[e] = 0u;
    }
}

// Widens the entry of `key` (false when its probe run is full).
__device__ __forceinline__ bool span_lds_add(SpanLds &L, uint32_t key, uint32_t zl, uint32_t zh)
{
    uint32_t h = (key * 2654435761u) >> (32 - 11);
#pragma unroll 1
    for (int p = 0; p < 8; ++p) {
        const uint32_t k = atomicCAS(&L.key[h], kSpanEmpty, key);
        if (k == kSpanEmpty || k == key) {
            atomicMin(&L.lo[h], zl);
            atomicMax(&L.hi[h], zh);
            return true;
        }
        h = (h + 1) & (kSpanLds - 1);
    }
    return false;
}

// One allocated block (pool slot) of the range pass.  Cell spans go to
// `emit(cell, zl, zh)`; tile spans and the near-plane stamp go to memory.
template <typename Emit>
__device__ __forceinline__ void range_block(const VolumeView &v, const Camera &cam, uint32_t stamp, int tiles_x,
                                            int tiles_y, uint32_t slot, Emit &&emit)
{
    uint32_t *tmin = v.tile_range;
    uint32_t *tmax = v.tile_range + (size_t)tiles_x * tiles_y;
    // camera axes in float: x_c = R^T (x - t)
    const float R[9] = {(float)cam.R[0], (float)cam.R[1], (float)cam.R[2], (float)cam.R[3], (float)cam.R[4],
                        (float)cam.R[5], (float)cam.R[6], (float)cam.R[7], (float)cam.R[8]};
    const float fx = (float)cam.fx, fy = (float)cam.fy, cx = (float)cam.cx, cy = (float)cam.cy;
    // a valid sample's stencil voxels are all non-chi, so its base voxel lies
    // in its block's box of non-chi voxels: q in [8B + lo, 8B + hi + 1] with
    // x = origin + (q + 1/2) voxel; a block without such voxels adds nothing
    const uint32_t box = v.block_box[slot];
    const uint32_t key = v.pool_keys[slot];
    if (!(box & kBoxValid) || key == kEmptyKey) return;   // no voxels, or a slot whose insertion failed
    int bx, by, bz;
    unpack_key(key, bx, by, bz);
    const float bwx = (float)((box_hi(box, 0) - box_lo(box, 0) + 1) * v.vs);
    const float bwy = (float)((box_hi(box, 1) - box_lo(box, 1) + 1) * v.vs);
    const float bwz = (float)((box_hi(box, 2) - box_lo(box, 2) + 1) * v.vs);
    // its min corner relative to the camera centre, in double then float
    const float ox = (float)(v.origin[0] + (8.0 * bx + box_lo(box, 0) + 0.5) * v.vs - cam.t[0]);
    const float oy = (float)(v.origin[1] + (8.0 * by + box_lo(box, 1) + 0.5) * v.vs - cam.t[1]);
    const float oz = (float)(v.origin[2] + (8.0 * bz + box_lo(box, 2) + 0.5) * v.vs - cam.t[2]);
    float zlo = 3.4e38f, zhi = -3.4e38f, ulo = 3.4e38f, uhi = -3.4e38f, vlo = 3.4e38f, vhi = -3.4e38f;
    bool behind = false;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const float dx = ox + ((k & 1) ? bwx : 0.0f), dy = oy + ((k & 2) ? bwy : 0.0f),
                    dz = oz + ((k & 4) ? bwz : 0.0f);
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
    if (zhi <= 0.0f) return;            // wholly behind the camera
    if (behind) {                         // reaches the camera plane: rays start at the camera
        v.state->near_stamp = stamp;
        return;
    }
    // pixel centres (i, j) inside the projected box; eps bounds the float
    // error of the projected corners (positions rounded to float relative to
    // the camera, then three products and a reciprocal)
    const float eps = 1e-5f * (fabsf(ulo - cx) + fabsf(uhi - cx) + fabsf(vlo - cy) + fabsf(vhi - cy) + fx + fy) +
                      1e-3f;
    const float ulo_e = fmaxf(ulo - eps, -1.0f), uhi_e = fminf(uhi + eps, (float)cam.width);
    const float vlo_e = fmaxf(vlo - eps, -1.0f), vhi_e = fminf(vhi + eps, (float)cam.height);
    const int i0 = max((int)ceilf(ulo_e), 0), i1 = min((int)floorf(uhi_e), cam.width - 1);
    const int j0 = max((int)ceilf(vlo_e), 0), j1 = min((int)floorf(vhi_e), cam.height - 1);
    if (!(ulo_e <= uhi_e && vlo_e <= vhi_e) || i0 > i1 || j0 > j1) return;
    const uint32_t zl = __float_as_uint(fmaxf(zlo * (1.0f - 1e-5f) - 1e-6f, 0.0f));
    const uint32_t zh = __float_as_uint(zhi * (1.0f + 1e-5f) + 1e-6f);
    const int c0 = i0 / kCell, c1 = i1 / kCell, d0 = j0 / kCell, d1 = j1 / kCell;
    if ((c1 - c0 + 1) * (d1 - d0 + 1) <= kCellFootprint) {
        // small footprint: widen the span of every cell it covers
        const int cw = (cam.width + kCell - 1) / kCell;
        for (int d = d0; d <= d1; ++d)
            for (int c = c0; c <= c1; ++c) emit((uint32_t)(d * cw + c), zl, zh);
        return;
    }
    // large footprint (blocks close to the camera): widen whole tiles
    for (int tj = j0 / kRT; tj <= j1 / kRT; ++tj)
        for (int ti = i0 / kRT; ti <= i1 / kRT; ++ti) {
            const size_t t = (size_t)tj * tiles_x + ti;
            if (tmin[t] > zl) atomicMin(&tmin[t], zl);
            if (tmax[t] < zh) atomicMax(&tmax[t], zh);
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

// Pool element offsets (slot * 512) of cell block B and its upper
// neighbours B + {0,1}^3; absent blocks point at the pool's chi block, so a
// stencil reaching them reads chi and is invalid without a branch.  Also
// whether every non-chi value in those 8 blocks is positive (then no sample
// of the cell can have F <= 0: F is a convex combination of them).
struct SlotCache {
    int B[3];
    uint32_t base[8];
    bool empty;      // block B itself is absent
    bool positive;
};

// Dense index: one load per neighbour; the entry carries the block's sign flag.
template <bool kDense>
__device__ __forceinline__ void fill_cache(const VolumeView &v, SlotCache &c, int bx, int by, int bz)
{
    c.B[0] = bx;
    c.B[1] = by;
    c.B[2] = bz;
    const uint32_t chi_base = v.capacity * (uint32_t)kBlockVoxels;
    bool pos = true;
    if constexpr (kDense) {
        // B itself is inside the grid (its stencils are); neighbours may not
        // be: those read B's own entry and are then taken as absent
        const uint32_t n0 = (uint32_t)v.nblk[0], n01 = n0 * (uint32_t)v.nblk[1];
        const uint32_t lin = (uint32_t)block_linear(v, bx, by, bz);
        const bool inx = bx + 1 < v.nblk[0], iny = by + 1 < v.nblk[1], inz = bz + 1 < v.nblk[2];
        int32_t raw[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool in = (!(k & 1) || inx) && (!(k & 2) || iny) && (!(k & 4) || inz);
            const uint32_t nb = lin + (in ? (k & 1) + ((k & 2) ? n0 : 0u) + ((k & 4) ? n01 : 0u) : 0u);
            raw[k] = v.block_index[nb];
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const bool in = (!(k & 1) || inx) && (!(k & 2) || iny) && (!(k & 4) || inz);
            const int32_t e = in ? raw[k] : -1;
            c.base[k] = e < 0 ? chi_base : (uint32_t)(e & kIndexSlotMask) * (uint32_t)kBlockVoxels;
            pos &= (e < 0) || (e & kIndexPositive);
            if (k == 0) c.empty = e < 0;
        }
    } else {
        uint32_t kmin = kKeyPosInf;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int x = bx + (k & 1), y = by + ((k >> 1) & 1), z = bz + ((k >> 2) & 1);
            int32_t sl = -1;
            if (x < v.nblk[0] && y < v.nblk[1] && z < v.nblk[2] && occupied(v, x, y, z))
                sl = hash_find(v, pack_key(x, y, z));
            c.base[k] = sl < 0 ? chi_base : (uint32_t)sl * (uint32_t)kBlockVoxels;
            if (sl >= 0) kmin = min(kmin, v.block_min[sl]);
            if (k == 0) c.empty = sl < 0;
        }
        pos = kmin > kKeyZero;
    }
    c.positive = pos;
}

// Trilinear F at integer base c (global voxel indices) with fractions f,
// using offsets from the cache (c must lie in cell c.B).  False when invalid.
template <typename S>
__device__ __forceinline__ bool interp_cached(const VolumeView &v, const SlotCache &cache, const int c[3],
                                              const float f[3], float &F)
{
    const S *__restrict__ pool = (const S *)v.poolT;
    const uint32_t l0 = c[0] & 7, l1 = c[1] & 7, l2 = c[2] & 7;
    // the stencil's upper neighbour leaves the block along an axis only from local index 7
    const bool cx = l0 == 7, cy = l1 == 7, cz = l2 == 7;
    const uint32_t x0 = l0, x1 = cx ? 0u : l0 + 1u;
    const uint32_t y0 = 8u * l1, y1 = cy ? 0u : y0 + 8u;
    const uint32_t z0 = 64u * l2, z1 = cz ? 0u : z0 + 64u;
    // block of each corner (x fastest): select along x, then y, then z
    const uint32_t *b = cache.base;
    const uint32_t b0 = b[0], b1 = cx ? b[1] : b0;
    const uint32_t b2 = cy ? b[2] : b0, b3 = cy ? (cx ? b[3] : b[2]) : b1;
    const uint32_t t45 = cx ? b[5] : b[4], t67 = cx ? b[7] : b[6];
    const uint32_t b4 = cz ? b[4] : b0, b5 = cz ? t45 : b1;
    const uint32_t b6 = cz ? (cy ? b[6] : b[4]) : b2, b7 = cz ? (cy ? t67 : t45) : b3;
    const float v0 = ld(pool + (b0 + x0 + y0 + z0)), v1 = ld(pool + (b1 + x1 + y0 + z0));
    const float v2 = ld(pool + (b2 + x0 + y1 + z0)), v3 = ld(pool + (b3 + x1 + y1 + z0));
    const float v4 = ld(pool + (b4 + x0 + y0 + z1)), v5 = ld(pool + (b5 + x1 + y0 + z1));
    const float v6 = ld(pool + (b6 + x0 + y1 + z1)), v7 = ld(pool + (b7 + x1 + y1 + z1));
    const float m = fmaxf(fmaxf(fmaxf(fabsf(v0), fabsf(v1)), fmaxf(fabsf(v2), fabsf(v3))),
                          fmaxf(fmaxf(fabsf(v4), fabsf(v5)), fmaxf(fabsf(v6), fabsf(v7))));
    const float x00 = v0 + f[0] * (v1 - v0);
    const float x10 = v2 + f[0] * (v3 - v2);
    const float x01 = v4 + f[0] * (v5 - v4);
    const float x11 = v6 + f[0] * (v7 - v6);
    const float y0f = x00 + f[1] * (x10 - x00);
    const float y1f = x01 + f[1] * (x11 - x01);
    F = y0f + f[2] * (y1f - y0f);
    return m <= 1.0f;
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
// samples before it all have their base voxel in B).  The division by h is a
// product with 1/h: the index found lies within one of the exit, and the
// test of its sample then returns the exit or one index before it (a later
// resume point is never returned).
__device__ __forceinline__ int cell_exit_sample(const Ray &r, const int B[3], double h, double inv_h)
{
    double s_exit = 1e300;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (r.dq[a] > 0.0) s_exit = fmin(s_exit, (8.0 * (B[a] + 1) - r.q0[a]) * r.inv[a]);
        else if (r.dq[a] < 0.0) s_exit = fmin(s_exit, (8.0 * B[a] - r.q0[a]) * r.inv[a]);
    }
    const int m = (int)fmin(floor(s_exit * inv_h), 2.0e9);
    double qm[3];
    q_at(r, (double)m * h, qm);
    const bool still = ((int)floor(qm[0]) >> 3) == B[0] && ((int)floor(qm[1]) >> 3) == B[1] &&
                       ((int)floor(qm[2]) >> 3) == B[2];
    return still ? m + 1 : m;
}

// Shuffle inside a group of G lanes: value of lane `src` of this lane's group.
template <int G>
__device__ __forceinline__ int group_lane(int lane, int src) { return (lane & ~(G - 1)) | src; }

// Thread `gt` of a launch space of (tiles x 64 rays x G lanes) for one frame.
// kMark: also set the bit of every block a march sample is based in (the
// footprint query; the timed raycast is instantiated without it).
template <typename S, int G, bool kDense, bool kMark = false>
__device__ __forceinline__ void raycast_body(const VolumeView &v, const Camera &cam, uint32_t stamp, int tiles_x,
                                             int tiles_y, float4 *__restrict__ vertex, float4 *__restrict__ normal,
                                             long long gt)
{
    static_assert(G >= 1 && G <= 16 && (G & (G - 1)) == 0, "group size");
    const int lane = threadIdx.x & 63;
    const int j = lane & (G - 1);                       // sample slot inside the ray's group
    // rays in 8x8-pixel tile order: 64 consecutive rays form one tile (the
    // launch covers fewer than 2^31 rays)
    const int ray = (int)(gt / G);
    const int tile = ray >> 6;
    const int within = ray & 63;
    const int ti = tile % tiles_x, tj = tile / tiles_x;
    // 16 consecutive rays cover one 4x4-pixel cell of the tile: they share
    // the cell's depth span and mostly the same blocks
    const int cq = within >> 4, k16 = within & 15;
    const int i = ti * kRT + (cq & 1) * 4 + (k16 & 3), jpix = tj * kRT + (cq >> 1) * 4 + (k16 >> 2);
    const bool active = tj < tiles_y && i < cam.width && jpix < cam.height;
    const double h = 0.5 * v.vs;

    Ray r;
#pragma unroll
    for (int a = 0; a < 3; ++a) r.q0[a] = r.dq[a] = r.inv[a] = r.d[a] = 0.0;
    int n_lo = 1, n_end = 0;   // sample indices (a ray crosses the grid in fewer than 2^31 samples)
    float zmin_t = 0.0f, zmax_t = -1.0f;
    bool near = false;
    if (active) {
        const size_t t = (size_t)tj * tiles_x + ti;
        // the pixel's cell span joined with its tile's (blocks with large footprints)
        const int cw = (cam.width + kCell - 1) / kCell, ch = (cam.height + kCell - 1) / kCell;
        const size_t cell = (size_t)(jpix / kCell) * cw + i / kCell;
        zmin_t = __uint_as_float(min(v.tile_range[t], v.pix_range[cell]));
        zmax_t =
            __uint_as_float(max(v.tile_range[(size_t)tiles_x * tiles_y + t], v.pix_range[(size_t)cw * ch + cell]));
        near = v.state->near_stamp == stamp;
    }
    // a ray with an empty span (and no block at the camera plane) misses
    // without a sample: the ray itself is only set up for the others
    if (active && (near || zmin_t <= zmax_t)) {
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
        if (!near) {   // the depth span (camera z = s / len along this ray)
            s_in = fmax(s_in, (double)zmin_t * len);
            s_out = fmin(s_out, (double)zmax_t * len);
        }
        if (!miss && s_in <= s_out) {
            n_lo = max((int)fmin(floor(s_in / h) - 1.0, 2.0e9), 1);
            n_end = (int)fmin(ceil(s_out / h) + 1.0, 2.0e9);
        }
    }

    // ---- march: the group evaluates samples n_base .. n_base + G - 1 per step.
    // An invalid sample carries F = NaN, so every comparison with it fails.
    const float kNaN = __builtin_nanf("");
    SlotCache cache;
    cache.B[0] = cache.B[1] = cache.B[2] = -(1 << 30);
#pragma unroll
    for (int k = 0; k < 8; ++k) cache.base[k] = v.capacity * (uint32_t)kBlockVoxels;   // the chi block
    cache.empty = true;
    cache.positive = false;
    const double inv_h = 2.0 * v.inv_vs;
    int n_base = n_lo;
    bool done = !(active && n_lo <= n_end);
    bool hit = false;
    float Fc = kNaN;     // carried last sample of the previous step
    double s_lo = 0.0, s_hi = 0.0;
    float F_lo = 0.0f, F_hi = 0.0f;
    while (__ballot(!done)) {
        const int n = n_base + j;
        double q[3];
        q_at(r, (double)n * h, q);
        int c[3];
        float f[3];
        const bool inside = stencil(v, q, c, f) && !done && n <= n_end;
        const int b0 = c[0] >> 3, b1 = c[1] >> 3, b2 = c[2] >> 3;
        const bool need = inside && (b0 != cache.B[0] || b1 != cache.B[1] || b2 != cache.B[2]);
        if (need) fill_cache<kDense>(v, cache, b0, b1, b2);
        if constexpr (kMark) {
            if (need && !cache.empty) {
                const uint64_t lb = block_linear(v, b0, b1, b2);
                atomicOr(&v.mark_bits[lb >> 5], 1u << (lb & 31));
            }
        }
        float F = kNaN;
        if (inside && !cache.empty) {
            float Fs;
            if (interp_cached<S>(v, cache, c, f, Fs)) F = Fs;
        }
        const uint32_t info = inside ? ((uint32_t)b0 | ((uint32_t)b1 << 10) | ((uint32_t)b2 << 20) |
                                        (cache.empty ? kInfoEmpty : (cache.positive ? kInfoPositive : 0u)))
                                     : 0u;
        // pair every sample with its predecessor (lane j - 1, or the carry)
        const float Fp_sh = __shfl(F, group_lane<G>(lane, (j + G - 1) & (G - 1)));
        const float Fp = j == 0 ? Fc : Fp_sh;
        const bool cross = !done && n <= n_end && Fp > 0.0f && F <= 0.0f;
        const unsigned long long m = __ballot(cross);
        const uint32_t gm = (uint32_t)(m >> (lane & ~(G - 1))) & ((G == 32 ? 0xffffffffu : (1u << G) - 1u));
        // (done and gm are the same in every lane of a group, so the group's
        // lanes all take part in these shuffles)
        if (!done && gm) {
            const int first = __builtin_ctz(gm);
            const int nh = n_base + first;
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
        const uint32_t info_last = (uint32_t)__shfl((int)info, group_lane<G>(lane, last));
        if (!done) {
            const int n_last = n_base + last;
            int next = n_last + 1;
            bool carry = true;
            if (n_last > n_end) {
                done = true;
            } else if (info_last & (kInfoEmpty | kInfoPositive)) {
                const int Bc[3] = {(int)(info_last & 1023u), (int)((info_last >> 10) & 1023u),
                                   (int)((info_last >> 20) & 1023u)};
                const int exit_n = cell_exit_sample(r, Bc, h, inv_h);   // first sample past the cell
                // empty: every sample before the exit is invalid; positive: none
                // before the cell's last sample can end a crossing
                const int target = (info_last & kInfoEmpty) ? exit_n : exit_n - 1;
                if (target > next) {
                    next = target;
                    carry = false;
                }
            }
            Fc = carry ? F_last : kNaN;
            n_base = next;
            if (n_base > n_end) done = true;
        }
    }

    // ---- refinement: quaternary search inside [s_lo, s_hi] (F_lo > 0 >= F_hi).
    // Each step samples the 3 inner quarter points (point m by lane m % G of
    // the group, in ceil(3 / G) rounds), so the points and hence the result do
    // not depend on the group size; 6 steps shrink the bracket 4096-fold.
    constexpr int kPts = 3, kSteps = 6, kRounds = (kPts + G - 1) / G;
    double a = s_lo, b = s_hi;
    float Fa = F_lo, Fb = F_hi;
    bool refine = hit;
    for (int it = 0; it < kSteps; ++it) {
        if (!__ballot(refine)) break;
        float Fp[kPts];
#pragma unroll
        for (int rd = 0; rd < kRounds; ++rd) {
            const int m = rd * G + j;
            float Fm = kNaN;
            if (refine && m < kPts) {
                double qm[3];
                q_at(r, a + (b - a) * (double)(m + 1) * 0.25, qm);
                float Fs;
                if (sample_q<S, kDense>(v, cache, qm, Fs)) Fm = Fs;
            }
#pragma unroll
            for (int mm = rd * G; mm < (rd + 1) * G && mm < kPts; ++mm)
                Fp[mm] = __shfl(Fm, group_lane<G>(lane, mm - rd * G));
        }
        if (refine) {
            bool bad = false;
            int k = kPts;   // first non-positive point: the root lies in (point k-1, point k]
#pragma unroll
            for (int mm = kPts - 1; mm >= 0; --mm) {
                bad |= Fp[mm] != Fp[mm];   // NaN: invalid
                if (Fp[mm] <= 0.0f) k = mm;
            }
            if (bad) {
                refine = false;   // an invalid point inside the bracket: keep the bracket
            } else {
                float F_km1 = Fa, F_k = Fb;
#pragma unroll
                for (int mm = 0; mm < kPts; ++mm) {
                    if (mm == k - 1) F_km1 = Fp[mm];
                    if (mm == k) F_k = Fp[mm];
                }
                const double na = k == 0 ? a : a + (b - a) * (double)k * 0.25;
                const double nb = k == kPts ? b : a + (b - a) * (double)(k + 1) * 0.25;
                Fa = F_km1;
                Fb = F_k;
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
#pragma unroll
        for (int e = 0; e < 6; ++e) Fs[e] = kNaN;
        // sample e in {+x, -x, +y, -y, +z, -z} is taken by lane e % G of the
        // group.  A lane taking several samples gives each its own copy of the
        // slot cache (the march's, refilled where the stencil leaves its
        // block), so their index and voxel loads are all in flight together.
        constexpr int kPer = (6 + G - 1) / G;
        int nc[kPer][3];
        float nf[kPer][3];
        bool nin[kPer];
        SlotCache ncache[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            const int e = j + t * G;
            nin[t] = hit && e < 6;
            if (nin[t]) {
                double qe[3] = {qh[0], qh[1], qh[2]};
                qe[e >> 1] += (e & 1) ? -1.0 : 1.0;
                nin[t] = stencil(v, qe, nc[t], nf[t]);
            }
            ncache[t] = cache;
            if (nin[t] && ((nc[t][0] >> 3) != cache.B[0] || (nc[t][1] >> 3) != cache.B[1] ||
                           (nc[t][2] >> 3) != cache.B[2]))
                fill_cache<kDense>(v, ncache[t], nc[t][0] >> 3, nc[t][1] >> 3, nc[t][2] >> 3);
        }
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            float Fv;
            if (nin[t] && interp_cached<S>(v, ncache[t], nc[t], nf[t], Fv)) {
#pragma unroll
                for (int e = 0; e < 6; ++e)
                    if (e == j + t * G) Fs[e] = Fv;
            }
        }
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            Fs[e] = __shfl(Fs[e], group_lane<G>(lane, e % G));
            ok = ok && Fs[e] == Fs[e];   // NaN: invalid
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

}  // namespace tsdf

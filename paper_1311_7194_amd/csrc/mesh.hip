// Marching-cubes extraction over the allocated blocks (Section 5: the
// polygonisation alternative to raycasting, in three stages: occupied cells
// and their output counts, a prefix sum into output offsets, polygonisation
// of the occupied cells only).
//
//   count   one workgroup per pool slot: the block's 9^3 corner tile (its own
//           512 voxels plus the x = 0 / y = 0 / z = 0 layers of its seven
//           +x/+y/+z neighbours) goes to LDS; each of the 512 lanes classifies
//           the cell whose low corner is its voxel; the workgroup sums the
//           triangle counts of its cells
//   scan    per tile of 1024 slots, an exclusive scan of the block counts;
//           then one workgroup scans the tile sums and writes the total
//   emit    blocks with triangles reload their tile; a workgroup scan over the
//           512 cells (in x + 8y + 64z order) places each cell's triangles
//           after the block's offset
//
// Cells: a cell spans the voxel centres g + {0,1}^3 and is valid when all
// eight hold a distance (|T_hat| <= 1) in allocated blocks inside the grid.
// Corner k (offset (k & 1, k >> 1 & 1, k >> 2 & 1)) is inside when F < 0.
// A crossed cell edge from voxel g along axis a carries one vertex, id
// 3 (gx + G0 (gy + G1 gz)) + a, at t = F(g) / (F(g) - F(g + e_a)).
//
// The case table is generated at compile time from this rule: on each cube
// face, walked counter-clockwise as seen from outside the cube, every
// crossing where the walk enters the inside corners is joined to the next
// crossing where it leaves them (so diagonal inside corners of an ambiguous
// face are cut off one by one, and the inside lies to the right of each
// segment seen from outside); the segments close into loops, and each loop,
// started at its smallest edge number, is fanned from that edge.  Cube edge
// 4a + m runs along axis a from the corner whose other two coordinates, in
// increasing axis order, are (m & 1, m >> 1).
#include <math.h>

#include "tsdf_internal.h"
#include "tsdf_mesh.h"

namespace tsdf {
namespace {

constexpr int kMcMaxTris = 5;

struct McTable {
    uint8_t ntri[256];
    uint8_t edge[256][3 * kMcMaxTris];
    bool overflow;   // a case needed more than kMcMaxTris triangles (rejected at compile time)
};

// Low corner of cube edge e (see the numbering above).
constexpr int mc_edge_lo(int e)
{
    const int a = e >> 2, m = e & 3;
    const int u = a == 0 ? 1 : 0, w = a == 2 ? 1 : 2;   // the other two axes, increasing
    return ((m & 1) << u) | ((m >> 1) << w);
}

// Cube edge joining corners p and q (which differ in one coordinate bit).
constexpr int mc_edge(int p, int q)
{
    const int d = p ^ q;
    const int a = d == 1 ? 0 : (d == 2 ? 1 : 2);
    const int lo = p & q;
    const int u = a == 0 ? 1 : 0, w = a == 2 ? 1 : 2;
    return 4 * a + ((lo >> u) & 1) + 2 * ((lo >> w) & 1);
}

constexpr McTable make_mc_table()
{
    McTable tab{};
    for (int c = 0; c < 256; ++c) {
        int next[12] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
        for (int a = 0; a < 3; ++a) {
            for (int side = 0; side < 2; ++side) {
                const int u = a == 0 ? 1 : 0, w = a == 2 ? 1 : 2;
                const int b = side << a;
                int ring[4] = {b, b | (1 << u), b | (1 << u) | (1 << w), b | (1 << w)};
                // the ring above turns counter-clockwise about +e_a for a = 0, 2 and
                // clockwise for a = 1 (e_u x e_w = -e_y); seen from outside the face
                // (normal (2 side - 1) e_a) reverse it where the two disagree
                const bool ccw_about_plus = a != 1;
                if (ccw_about_plus != (side == 1)) {
                    const int t = ring[1];
                    ring[1] = ring[3];
                    ring[3] = t;
                }
                for (int k = 0; k < 4; ++k) {
                    const bool in_k = (c >> ring[k]) & 1, in_k1 = (c >> ring[(k + 1) & 3]) & 1;
                    if (in_k || !in_k1) continue;   // not an entering crossing
                    int j = (k + 1) & 3;
                    while (!(((c >> ring[j]) & 1) && !((c >> ring[(j + 1) & 3]) & 1))) j = (j + 1) & 3;
                    next[mc_edge(ring[k], ring[(k + 1) & 3])] = mc_edge(ring[j], ring[(j + 1) & 3]);
                }
            }
        }
        bool seen[12] = {};
        int nt = 0;
        for (int e0 = 0; e0 < 12; ++e0) {
            if (next[e0] < 0 || seen[e0]) continue;
            int loop[12] = {};
            int len = 0;
            for (int e = e0; !seen[e]; e = next[e]) {
                seen[e] = true;
                loop[len++] = e;
            }
            for (int i = 1; i + 1 < len; ++i) {
                if (nt == kMcMaxTris) {
                    tab.overflow = true;
                    break;
                }
                tab.edge[c][3 * nt + 0] = (uint8_t)loop[0];
                tab.edge[c][3 * nt + 1] = (uint8_t)loop[i];
                tab.edge[c][3 * nt + 2] = (uint8_t)loop[i + 1];
                ++nt;
            }
        }
        tab.ntri[c] = (uint8_t)nt;
    }
    return tab;
}

constexpr McTable kMcTableHost = make_mc_table();
static_assert(!kMcTableHost.overflow, "marching-cubes case with more than kMcMaxTris triangles");
static_assert(kMcTableHost.ntri[0] == 0 && kMcTableHost.ntri[255] == 0 && kMcTableHost.ntri[1] == 1,
              "marching-cubes table");

__constant__ McTable kMcTable = kMcTableHost;

constexpr int kMcLanes = 64;         // one wavefront per block: lane (x, y) takes the cells of its z column
constexpr int kTile = 9;             // corner tile edge
constexpr int kHalo = 217;           // 3 * 64 + 3 * 8 + 1 neighbour values
constexpr uint32_t kMcGrid = 16384;  // single-wavefront workgroups striding over the pool
constexpr uint32_t kScanTile = 1024; // slots per first-level scan tile
constexpr int kOwnerChunk = 1024;    // output triangles of a block placed per round

template <typename S>
__device__ __forceinline__ float mc_load(const S *p);
template <>
__device__ __forceinline__ float mc_load<float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float mc_load<__half>(const __half *p) { return __half2float(*p); }

struct McLds {
    float f[kTile * kTile * kTile];   // corner tile, x fastest
    int32_t nslot[8];                 // pool slots of the +x/+y/+z neighbours (-1: none)
    uint8_t cases[kBlockVoxels];      // case of each cell (0 when invalid)
    uint16_t owner[kOwnerChunk];      // emit: cell | triangle << 9 of each output triangle of a round
};

__device__ __forceinline__ int tidx(int x, int y, int z) { return x + kTile * y + kTile * kTile * z; }

// Fills L.f with the corner tile of the block in `slot` (key `key`): chi
// where a neighbour block is unallocated or outside the grid.  Ends with a
// barrier (of the one-wavefront workgroup).
template <typename S>
__device__ void load_tile(const VolumeView &v, uint32_t slot, uint32_t key, McLds &L)
{
    const int t = threadIdx.x;
    int bx, by, bz;
    unpack_key(key, bx, by, bz);
    if (t >= 1 && t < 8) {
        const int nx = bx + (t & 1), ny = by + ((t >> 1) & 1), nz = bz + (t >> 2);
        int32_t s = -1;
        if (nx < v.nblk[0] && ny < v.nblk[1] && nz < v.nblk[2]) {
            if (v.block_index) {
                const int32_t e = v.block_index[block_linear(v, nx, ny, nz)];
                s = e < 0 ? -1 : (e & kIndexSlotMask);
            } else {
                s = hash_find(v, pack_key(nx, ny, nz));
            }
        }
        L.nslot[t] = s;
    }
    const S *T = (const S *)v.poolT + (size_t)slot * kBlockVoxels;
    float own[8];
#pragma unroll
    for (int z = 0; z < 8; ++z) own[z] = mc_load<S>(T + t + 64 * z);   // 64 consecutive voxels per z
#pragma unroll
    for (int z = 0; z < 8; ++z) L.f[tidx(t & 7, t >> 3, z)] = own[z];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int h = t + 64 * r;
        if (h < kHalo) {
            int n, lx = 0, ly = 0, lz = 0;   // neighbour (bits x, y, z) and its voxel
            if (h < 64) {
                n = 1, ly = h & 7, lz = h >> 3;
            } else if (h < 128) {
                n = 2, lx = h & 7, lz = (h >> 3) & 7;
            } else if (h < 192) {
                n = 4, lx = h & 7, ly = (h >> 3) & 7;
            } else if (h < 200) {
                n = 3, lz = h - 192;
            } else if (h < 208) {
                n = 5, ly = h - 200;
            } else if (h < 216) {
                n = 6, lx = h - 208;
            } else {
                n = 7;
            }
            const int32_t s = L.nslot[n];
            const float val = s < 0 ? kChi : mc_load<S>((const S *)v.poolT + (size_t)s * kBlockVoxels + lx + 8 * ly + 64 * lz);
            L.f[tidx((n & 1) ? 8 : lx, (n & 2) ? 8 : ly, (n & 4) ? 8 : lz)] = val;
        }
    }
    __syncthreads();
}

// Cases of the eight cells of this lane's column (cell x + 8y + 64z, z = 0..7;
// 0 when a corner is not a distance), walking up the column so that each
// z-layer of corners is read once.
__device__ __forceinline__ void column_cases(const McLds &L, int cs[8])
{
    const int t = threadIdx.x, x = t & 7, y = t >> 3;
    float lo[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) lo[k] = L.f[tidx(x + (k & 1), y + (k >> 1), 0)];
#pragma unroll
    for (int z = 0; z < 8; ++z) {
        float hi[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) hi[k] = L.f[tidx(x + (k & 1), y + (k >> 1), z + 1)];
        bool ok = true;
        int c = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            ok = ok && fabsf(lo[k]) <= 1.0f && fabsf(hi[k]) <= 1.0f;
            c |= (lo[k] < 0.0f ? 1 : 0) << k;
            c |= (hi[k] < 0.0f ? 1 : 0) << (k + 4);
        }
        cs[z] = ok ? c : 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) lo[k] = hi[k];
    }
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += (uint32_t)__shfl_xor((int)x, off);
    return x;
}

__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, off);
        if (lane >= off) x += y;
    }
    return x;
}

template <typename S>
__global__ __launch_bounds__(kMcLanes) void mc_count_kernel(VolumeView v, uint32_t *__restrict__ counts)
{
    __shared__ McLds L;
    const uint32_t n = min(v.state->pool_count, v.capacity);
    for (uint32_t slot = blockIdx.x; slot < n; slot += gridDim.x) {
        const uint32_t key = v.pool_keys[slot];
        if (key == kEmptyKey) {   // a slot whose insertion failed holds no block
            if (threadIdx.x == 0) counts[slot] = 0;
            continue;
        }
        load_tile<S>(v, slot, key, L);
        int cs[8];
        column_cases(L, cs);
        uint32_t nt = 0;
#pragma unroll
        for (int z = 0; z < 8; ++z) nt += kMcTable.ntri[cs[z]];
        nt = wave_sum(nt);
        if (threadIdx.x == 0) counts[slot] = nt;
        __syncthreads();   // the next block's tile overwrites this one
    }
}

// Exclusive scan of counts within each tile of kScanTile slots (256 lanes x
// 4 slots); tile sums to tile_sum.
__global__ __launch_bounds__(256) void mc_scan_tiles_kernel(const VolumeView v, const uint32_t *__restrict__ counts,
                                                            uint32_t *__restrict__ offsets,
                                                            uint32_t *__restrict__ tile_sum)
{
    __shared__ uint32_t wtot[4];
    const uint32_t n = min(v.state->pool_count, v.capacity);
    const uint32_t base = blockIdx.x * kScanTile;
    if (base >= n) return;   // uniform over the workgroup
    const uint32_t i0 = base + 4 * threadIdx.x;
    uint32_t c[4], s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        c[k] = i0 + k < n ? counts[i0 + k] : 0u;
        s += c[k];
    }
    const uint32_t inc = wave_inclusive_scan(s);
    const int wave = threadIdx.x >> 6;
    if (__lane_id() == 63) wtot[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wtot[w];
    uint32_t run = before + inc - s;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (i0 + k < n) offsets[i0 + k] = run;
        run += c[k];
    }
    if (threadIdx.x == 255) tile_sum[blockIdx.x] = run;
}

// One workgroup: exclusive scan of the tile sums into tile_base; the total
// triangle count to *count.
__global__ __launch_bounds__(1024) void mc_scan_top_kernel(const VolumeView v, const uint32_t *__restrict__ tile_sum,
                                                           unsigned long long *__restrict__ tile_base,
                                                           unsigned long long *__restrict__ count)
{
    __shared__ unsigned long long wtot[16];
    __shared__ unsigned long long carry;
    const uint32_t n = min(v.state->pool_count, v.capacity);
    const uint32_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = __lane_id();
    for (uint32_t b = 0; b < ntiles; b += 1024) {
        const uint32_t i = b + threadIdx.x;
        unsigned long long x = i < ntiles ? tile_sum[i] : 0ull;
        unsigned long long inc = x;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned long long y = __shfl_up(inc, off);
            if (lane >= off) inc += y;
        }
        if (lane == 63) wtot[wave] = inc;
        __syncthreads();
        unsigned long long before = carry;
        for (int w = 0; w < wave; ++w) before += wtot[w];
        if (i < ntiles) tile_base[i] = before + inc - x;
        __syncthreads();
        if (threadIdx.x == 1023) carry = before + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = carry;
}

// Emit: the block's triangles are placed in rounds of kOwnerChunk; in each
// round every cell writes, for each of its triangles in the round, its cell
// and triangle number into `owner` at the triangle's position, then lane k
// computes and writes the round's triangles k, k + 64, ... (consecutive
// lanes write consecutive triangles).
template <typename S>
__global__ __launch_bounds__(kMcLanes) void mc_emit_kernel(VolumeView v, const uint32_t *__restrict__ counts,
                                                           const uint32_t *__restrict__ offsets,
                                                           const unsigned long long *__restrict__ tile_base,
                                                           unsigned long long cap, long long *__restrict__ vid,
                                                           float *__restrict__ tpar, float *__restrict__ xyz)
{
    __shared__ McLds L;
    const uint32_t n = min(v.state->pool_count, v.capacity);
    const int t = threadIdx.x;
    const long long G0 = v.dims[0], G1 = v.dims[1];
    for (uint32_t slot = blockIdx.x; slot < n; slot += gridDim.x) {
        const uint32_t total = counts[slot];
        if (total == 0) continue;   // uniform: no triangles (or no block) in this slot
        const unsigned long long base = tile_base[slot / kScanTile] + offsets[slot];
        if (base >= cap) continue;
        const uint32_t key = v.pool_keys[slot];
        load_tile<S>(v, slot, key, L);
        int cs[8];
        column_cases(L, cs);
        // exclusive prefix of the triangle counts in cell order (x + 8y + 64z)
        uint32_t pre[8], run = 0;
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            L.cases[t + 64 * z] = (uint8_t)cs[z];
            const uint32_t nt = kMcTable.ntri[cs[z]];
            const uint32_t inc = wave_inclusive_scan(nt);
            pre[z] = run + inc - nt;
            run += (uint32_t)__shfl((int)inc, 63);
        }
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        for (uint32_t r0 = 0; r0 < total; r0 += kOwnerChunk) {
#pragma unroll
            for (int z = 0; z < 8; ++z) {
                const uint32_t nt = kMcTable.ntri[cs[z]];
                for (uint32_t i = 0; i < nt; ++i) {
                    const uint32_t k = pre[z] + i;
                    if (k >= r0 && k < r0 + kOwnerChunk) L.owner[k - r0] = (uint16_t)((t + 64 * z) | (i << 9));
                }
            }
            __syncthreads();
            const uint32_t r1 = min(total, r0 + (uint32_t)kOwnerChunk);
            for (uint32_t k = r0 + t; k < r1; k += kMcLanes) {
                const unsigned long long o = base + k;
                if (o >= cap) break;
                const uint32_t e = L.owner[k - r0];
                const int cell = (int)(e & 511u), i = (int)(e >> 9);
                const int c = L.cases[cell];
                const int cx = cell & 7, cy = (cell >> 3) & 7, cz = cell >> 6;
                const long long gx = 8 * bx + cx, gy = 8 * by + cy, gz = 8 * bz + cz;
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const int ed = kMcTable.edge[c][3 * i + j];
                    const int a = ed >> 2, lo = mc_edge_lo(ed), hi = lo | (1 << a);
                    const float flo = L.f[tidx(cx + (lo & 1), cy + ((lo >> 1) & 1), cz + (lo >> 2))];
                    const float fhi = L.f[tidx(cx + (hi & 1), cy + ((hi >> 1) & 1), cz + (hi >> 2))];
                    const float te = flo / (flo - fhi);
                    const long long px = gx + (lo & 1), py = gy + ((lo >> 1) & 1), pz = gz + (lo >> 2);
                    vid[3 * o + j] = 3 * (px + G0 * (py + G1 * pz)) + a;
                    tpar[3 * o + j] = te;
                    if (xyz) {
                        const double p[3] = {(double)px + 0.5 + (a == 0 ? (double)te : 0.0),
                                             (double)py + 0.5 + (a == 1 ? (double)te : 0.0),
                                             (double)pz + 0.5 + (a == 2 ? (double)te : 0.0)};
#pragma unroll
                        for (int q = 0; q < 3; ++q) xyz[9 * o + 3 * j + q] = (float)(v.origin[q] + p[q] * v.vs);
                    }
                }
            }
            __syncthreads();
        }
    }
}

struct MeshWork {
    uint32_t *counts, *offsets, *tile_sum;
    unsigned long long *tile_base;
    uint64_t bytes;
};

uint64_t align256(uint64_t b) { return (b + 255) & ~(uint64_t)255; }

MeshWork mesh_work(const VolumeView &v, void *base)
{
    const uint64_t cap = v.capacity, tiles = (cap + kScanTile - 1) / kScanTile;
    MeshWork w{};
    uint8_t *p = (uint8_t *)base;
    w.counts = (uint32_t *)p;
    p += align256(4 * cap);
    w.offsets = (uint32_t *)p;
    p += align256(4 * cap);
    w.tile_sum = (uint32_t *)p;
    p += align256(4 * tiles);
    w.tile_base = (unsigned long long *)p;
    p += align256(8 * tiles);
    w.bytes = (uint64_t)(p - (uint8_t *)base);
    return w;
}

}  // namespace
}  // namespace tsdf

using namespace tsdf;

extern "C" {

int32_t tsdf_mesh_case(int32_t c, int32_t edges[15])
{
    if (c < 0 || c > 255 || !edges) return -1;
    for (int i = 0; i < 15; ++i) edges[i] = i < 3 * kMcTableHost.ntri[c] ? kMcTableHost.edge[c][i] : -1;
    return kMcTableHost.ntri[c];
}

uint64_t tsdf_mesh_workspace_bytes(const tsdf_volume *vol)
{
    if (!vol) return 0;
    return mesh_work(volume_view(vol), nullptr).bytes;
}

tsdf_status tsdf_extract_mesh(tsdf_volume *vol, int64_t *vertex_id_dev, float *t_dev, float *xyz_dev, uint64_t cap,
                              void *work_dev, uint64_t work_bytes, uint64_t *count_dev, hipStream_t stream)
{
    if (!vol || !count_dev || !work_dev || work_bytes < tsdf_mesh_workspace_bytes(vol) ||
        (cap > 0 && (!vertex_id_dev || !t_dev)))
        return TSDF_EINVAL;
    const tsdf_status st = volume_enqueue(vol, stream, nullptr);
    if (st != TSDF_OK) return st;
    const VolumeView v = volume_view(vol);
    const MeshWork w = mesh_work(v, work_dev);
    const uint32_t tiles = (v.capacity + kScanTile - 1) / kScanTile;
    const bool f16 = v.storage == TSDF_F16;
    if (f16)
        hipLaunchKernelGGL(mc_count_kernel<__half>, dim3(kMcGrid), dim3(kMcLanes), 0, stream, v, w.counts);
    else
        hipLaunchKernelGGL(mc_count_kernel<float>, dim3(kMcGrid), dim3(kMcLanes), 0, stream, v, w.counts);
    hipLaunchKernelGGL(mc_scan_tiles_kernel, dim3(tiles), dim3(256), 0, stream, v, w.counts, w.offsets, w.tile_sum);
    hipLaunchKernelGGL(mc_scan_top_kernel, dim3(1), dim3(1024), 0, stream, v, w.tile_sum, w.tile_base,
                       (unsigned long long *)count_dev);
    if (cap > 0) {
        if (f16)
            hipLaunchKernelGGL(mc_emit_kernel<__half>, dim3(kMcGrid), dim3(kMcLanes), 0, stream, v, w.counts,
                               w.offsets, w.tile_base, (unsigned long long)cap, (long long *)vertex_id_dev, t_dev,
                               xyz_dev);
        else
            hipLaunchKernelGGL(mc_emit_kernel<float>, dim3(kMcGrid), dim3(kMcLanes), 0, stream, v, w.counts,
                               w.offsets, w.tile_base, (unsigned long long)cap, (long long *)vertex_id_dev, t_dev,
                               xyz_dev);
    }
    return hipGetLastError() == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

}  // extern "C"

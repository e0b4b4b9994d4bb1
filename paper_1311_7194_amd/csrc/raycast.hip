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
// of occupied blocks.  Here a compute pass does the same at the granularity
// of 4x4-pixel cells: for every allocated block it projects the box of
// stencil bases that can give a valid sample (the bounding box of the
// block's non-chi voxels, extended by one voxel upwards) and widens the
// [min, max] camera depth of every cell holding a pixel centre the box's
// projection may cover (boxes whose projection spans more than 64 cells
// widen whole 8x8-pixel tiles instead).  Every valid sample lies in such a
// box, so starting and ending each ray at its cell's span (joined with its
// tile's) skips only invalid samples.
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
#include "raycast_device.h"

namespace tsdf {

__global__ void range_clear_kernel(VolumeView v, int tiles_x, int tiles_y, int width, int height)
{
    range_clear_body(v, tiles_x, tiles_y, width, height, (long long)blockIdx.x * blockDim.x + threadIdx.x);
}

__global__ __launch_bounds__(256) void range_kernel(VolumeView v, Camera cam, uint32_t stamp, int tiles_x,
                                                    int tiles_y)
{
    __shared__ SpanLds L;
    span_lds_init(L);
    __syncthreads();
    const int cw = (cam.width + kCell - 1) / kCell, ch = (cam.height + kCell - 1) / kCell;
    uint32_t *cmin = v.pix_range, *cmax = v.pix_range + (size_t)cw * ch;
    const uint32_t n = min(v.state->pool_count, v.capacity);
    for (uint32_t slot = blockIdx.x * 256u + threadIdx.x; slot < n; slot += gridDim.x * 256u)
        range_block(v, cam, stamp, tiles_x, tiles_y, slot, [&](uint32_t c, uint32_t zl, uint32_t zh) {
            if (!span_lds_add(L, c, zl, zh)) {
                atomicMin(&cmin[c], zl);   // no return value: the lane does not wait
                atomicMax(&cmax[c], zh);
            }
        });
    __syncthreads();
    for (int e = threadIdx.x; e < kSpanLds; e += 256) {
        const uint32_t c = L.key[e];
        if (c != kSpanEmpty) {
            atomicMin(&cmin[c], L.lo[e]);
            atomicMax(&cmax[c], L.hi[e]);
        }
    }
}

// One wavefront per workgroup: march lengths differ widely between
// wavefronts (most rays of a frame march little or not at all), and a CU
// takes a new workgroup only where all of its wavefronts fit, so single-wave
// workgroups keep the SIMDs fuller (1280x960 hand sequence: 141 -> 124 us
// at 4 lanes per ray; 640x480 orbit: 284 -> 246 us, now at 8 lanes per ray).
constexpr int kRayWG = 64;

template <typename S, int G, bool kDense, bool kMark = false>
__global__ __launch_bounds__(kRayWG) void raycast_kernel(VolumeView v, Camera cam, uint32_t stamp, int tiles_x,
                                                      int tiles_y, float4 *__restrict__ vertex,
                                                      float4 *__restrict__ normal)
{
    // Workgroups are dealt to the 8 XCDs in turn.  With up to 4 lanes per ray
    // the G wavefronts of a tile go to one XCD, where they read the same
    // blocks through its L2, and neighbouring tiles to different ones (the
    // grid is then a multiple of 8 G): 124 -> 120 us on the 1280x960 hand
    // sequence at 4 lanes.  At 8 lanes the plain order measured faster.
    uint32_t wg = blockIdx.x;
    if constexpr (G <= 4) {
        const uint32_t grp = blockIdx.x / (8u * G), r = blockIdx.x % (8u * G);
        wg = grp * (8u * G) + (r & 7u) * G + (r >> 3);
    }
    raycast_body<S, G, kDense, kMark>(v, cam, stamp, tiles_x, tiles_y, vertex, normal,
                               (long long)wg * kRayWG + threadIdx.x);
}

template <typename S, bool kDense, bool kMark>
static void launch_group(int G, dim3 grid, hipStream_t s, const VolumeView &v, const Camera &cam, uint32_t stamp,
                         int tx, int ty, float4 *vertex, float4 *normal)
{
    switch (G) {
    case 1: hipLaunchKernelGGL((raycast_kernel<S, 1, kDense, kMark>), grid, dim3(kRayWG), 0, s, v, cam, stamp, tx, ty, vertex, normal); break;
    case 2: hipLaunchKernelGGL((raycast_kernel<S, 2, kDense, kMark>), grid, dim3(kRayWG), 0, s, v, cam, stamp, tx, ty, vertex, normal); break;
    case 4: hipLaunchKernelGGL((raycast_kernel<S, 4, kDense, kMark>), grid, dim3(kRayWG), 0, s, v, cam, stamp, tx, ty, vertex, normal); break;
    case 16: hipLaunchKernelGGL((raycast_kernel<S, 16, kDense, kMark>), grid, dim3(kRayWG), 0, s, v, cam, stamp, tx, ty, vertex, normal); break;
    default: hipLaunchKernelGGL((raycast_kernel<S, 8, kDense, kMark>), grid, dim3(kRayWG), 0, s, v, cam, stamp, tx, ty, vertex, normal); break;
    }
}

template <typename S, bool kDense>
static void launch_group(bool mark, int G, dim3 grid, hipStream_t s, const VolumeView &v, const Camera &cam,
                         uint32_t stamp, int tx, int ty, float4 *vertex, float4 *normal)
{
    if (mark) launch_group<S, kDense, true>(G, grid, s, v, cam, stamp, tx, ty, vertex, normal);
    else launch_group<S, kDense, false>(G, grid, s, v, cam, stamp, tx, ty, vertex, normal);
}

hipError_t launch_range(const VolumeView &v, const Camera &cam, uint32_t stamp, hipStream_t s)
{
    const int tiles_x = (cam.width + kRT - 1) / kRT, tiles_y = (cam.height + kRT - 1) / kRT;
    const int n_tiles = tiles_x * tiles_y;
    hipLaunchKernelGGL(range_clear_kernel, dim3((n_tiles * 64 + 255) / 256), dim3(256), 0, s, v, tiles_x, tiles_y,
                       cam.width, cam.height);
    // range pass over the allocated blocks (grid-stride; the block count stays on the device)
    hipLaunchKernelGGL(range_kernel, dim3(2048), dim3(256), 0, s, v, cam, stamp, tiles_x, tiles_y);
    return hipGetLastError();
}

hipError_t launch_march(const VolumeView &v, const Camera &cam, uint32_t stamp, int group, float4 *vertex,
                        float4 *normal, hipStream_t s, bool mark)
{
    const int tiles_x = (cam.width + kRT - 1) / kRT, tiles_y = (cam.height + kRT - 1) / kRT;
    const int G = (group == 1 || group == 2 || group == 4 || group == 16) ? group : 8;
    const long long threads = (long long)tiles_x * tiles_y * 64 * G;
    const long long unit = (G <= 4 ? 8LL * G : 1LL) * kRayWG;   // whole groups of 8 tiles' wavefronts
    dim3 grid((unsigned)((threads + unit - 1) / unit * (unit / kRayWG)));
    const bool dense = v.block_index != nullptr;
    if (v.storage == TSDF_F16) {
        if (dense) launch_group<__half, true>(mark, G, grid, s, v, cam, stamp, tiles_x, tiles_y, vertex, normal);
        else launch_group<__half, false>(mark, G, grid, s, v, cam, stamp, tiles_x, tiles_y, vertex, normal);
    } else {
        if (dense) launch_group<float, true>(mark, G, grid, s, v, cam, stamp, tiles_x, tiles_y, vertex, normal);
        else launch_group<float, false>(mark, G, grid, s, v, cam, stamp, tiles_x, tiles_y, vertex, normal);
    }
    return hipGetLastError();
}

// Number of set bits of a bitmap, added to the device state's footprint field.
__global__ __launch_bounds__(256) void count_bits_kernel(const uint32_t *__restrict__ bits, uint64_t words,
                                                         unsigned long long *__restrict__ out)
{
    unsigned long long c = 0;
    for (uint64_t w = (uint64_t)blockIdx.x * 256 + threadIdx.x; w < words; w += (uint64_t)gridDim.x * 256)
        c += (unsigned long long)__popc(bits[w]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}

hipError_t launch_count_bits(const uint32_t *bits, uint64_t words, unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(count_bits_kernel, dim3(1024), dim3(256), 0, s, bits, words, out);
    return hipGetLastError();
}

}  // namespace tsdf

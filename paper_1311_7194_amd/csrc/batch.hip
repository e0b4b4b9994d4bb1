// Batched multi-scene step: fusion and raycast of several independent
// volumes, one frame each, in six launches that cover every scene (frame
// reset, pixel preparation, persistent block fusion over all scenes'
// candidates, range reset, persistent range pass over all scenes' blocks,
// raycast).  The sequence can be captured once into a hipGraph and replayed
// every step; per-step inputs (depth maps, poses, output maps, which scenes
// have a frame) live in a device table uploaded before each replay.
// Every scene runs exactly the kernel bodies of the single-volume path, so
// its results are identical to fusing and raycasting it alone.
#include <string.h>

#include <new>
#include <vector>

#include <hip/hip_cooperative_groups.h>

#include "fuse_device.h"
#include "raycast_device.h"
#include "tsdf_batch.h"

namespace tsdf {

constexpr int kMaxScenes = 64;

struct SceneDesc {
    VolumeView v;
    Camera cam;
    FuseCam fc;
    NoiseParams noise;
    const float *depth;
    float4 *vertex;
    float4 *normal;
    uint32_t active;
    uint32_t stamp;
    int32_t tiles_x8, tiles_y8;     // raycast tiles
    int32_t tiles_x16, tiles_y16;   // preparation tiles
    uint32_t prep_base;             // first preparation workgroup of this scene
    uint32_t ray_base;              // first raycast tile of this scene
};

__device__ __forceinline__ int scene_of(const SceneDesc *__restrict__ sd, int n, uint32_t idx, bool ray)
{
    int s = 0;
    for (int k = 1; k < n; ++k)
        if ((ray ? sd[k].ray_base : sd[k].prep_base) <= idx) s = k;
    return s;
}

__global__ void batch_frame_begin(const SceneDesc *__restrict__ sd)
{
    const SceneDesc &d = sd[blockIdx.x];
    if (d.active) frame_begin_body(d.v.state, d.v.ctr, threadIdx.x);
}

template <bool kMlp>
__global__ __launch_bounds__(256) void batch_prep(const SceneDesc *__restrict__ sd, int n)
{
    const int s = scene_of(sd, n, blockIdx.x, false);
    const SceneDesc &d = sd[s];
    if (!d.active) return;   // the whole workgroup leaves together
    const uint32_t local = blockIdx.x - d.prep_base;
    prep_body<kMlp>(d.v, d.depth, d.cam, d.noise, (int)(local % (uint32_t)d.tiles_x16),
                    (int)(local / (uint32_t)d.tiles_x16));
}

// Offsets of each scene's share in a concatenation of per-scene counts
// (candidates or allocated blocks), computed once per workgroup into LDS.
template <bool kBlocks>
__device__ __forceinline__ void scene_prefix(const SceneDesc *__restrict__ sd, int n, uint32_t *pre)
{
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        pre[0] = 0;
        for (int k = 0; k < n; ++k) {
            const VolumeView &v = sd[k].v;
            const uint32_t c = !sd[k].active ? 0u
                               : kBlocks    ? min(v.state->pool_count, v.capacity)
                                            : min(v.state->cand_count, v.max_candidates);
            acc += c;
            pre[k + 1] = acc;
        }
    }
    __syncthreads();
}

// Scene whose share of the concatenation holds position g (wave-uniform g).
__device__ __forceinline__ int scene_at(const uint32_t *pre, int n, uint32_t g)
{
    int s = 0;
    for (int k = 1; k < n; ++k) s += pre[k] <= g ? 1 : 0;
    return __builtin_amdgcn_readfirstlane(s);
}

// Persistent fusion over the concatenation of every active scene's candidates;
// a wavefront's counts go to a scene's counters when it moves on to the next.
template <typename S>
// five waves per SIMD: a few spilled registers cost less than the lost latency hiding
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void batch_fuse(const SceneDesc *__restrict__ sd, int n)
{
    __shared__ uint32_t pre[kMaxScenes + 1];
    scene_prefix<false>(sd, n, pre);
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (threadIdx.x >> 6));
    const uint32_t nwaves = gridDim.x * 4u;
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)n && sd[threadIdx.x].active)
        atomicAdd(&sd[threadIdx.x].v.state->total_candidates,
                  (unsigned long long)(pre[threadIdx.x + 1] - pre[threadIdx.x]));
    FuseAcc acc;
    int cur = -1;
    for (uint32_t g = wave; g < pre[n]; g += nwaves) {
        const int s = scene_at(pre, n, g);
        if (s != cur) {
            if (cur >= 0) fuse_flush(sd[cur].v, acc, wave, lane);
            cur = s;
        }
        const SceneDesc &d = sd[s];
        fuse_block<S>(d.v, d.cam, d.fc, d.v.cand_list[g - pre[s]], lane, acc);
    }
    if (cur >= 0) fuse_flush(sd[cur].v, acc, wave, lane);
}

// One thread per (tile, pixel slot) of every scene's raycast tiles.
__global__ void batch_range_clear(const SceneDesc *__restrict__ sd, int n, uint32_t total_tiles)
{
    const long long gt = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t tile = (uint32_t)(gt >> 6);
    if (tile >= total_tiles) return;
    const SceneDesc &d = sd[scene_of(sd, n, tile, true)];
    if (!d.active) return;
    range_clear_body(d.v, d.tiles_x8, d.tiles_y8, d.cam.width, d.cam.height, gt - (long long)d.ray_base * 64);
}

// Persistent range pass over the concatenation of every active scene's blocks.
__global__ __launch_bounds__(256) void batch_range(const SceneDesc *__restrict__ sd, int n)
{
    __shared__ uint32_t pre[kMaxScenes + 1];
    __shared__ SpanLds L;
    span_lds_init(L);
    scene_prefix<true>(sd, n, pre);   // (synchronises the workgroup)
    for (uint32_t g = blockIdx.x * 256u + threadIdx.x; g < pre[n]; g += gridDim.x * 256u) {
        int s = 0;
        for (int k = 1; k < n; ++k) s += pre[k] <= g ? 1 : 0;
        const SceneDesc &d = sd[s];
        range_block(d.v, d.cam, d.stamp, d.tiles_x8, d.tiles_y8, g - pre[s],
                    [&](uint32_t c, uint32_t zl, uint32_t zh) {
                        if (!span_lds_add(L, ((uint32_t)s << 26) | c, zl, zh)) {
                            uint32_t *cmin = d.v.pix_range;
                            uint32_t *cmax = cmin + (size_t)((d.cam.width + kCell - 1) / kCell) *
                                                        ((d.cam.height + kCell - 1) / kCell);
                            atomicMin(&cmin[c], zl);
                            atomicMax(&cmax[c], zh);
                        }
                    });
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kSpanLds; e += 256) {
        const uint32_t key = L.key[e];
        if (key != kSpanEmpty) {
            const SceneDesc &d = sd[key >> 26];
            const uint32_t c = key & ((1u << 26) - 1u);
            uint32_t *cmin = d.v.pix_range;
            uint32_t *cmax = cmin + (size_t)((d.cam.width + kCell - 1) / kCell) * ((d.cam.height + kCell - 1) / kCell);
            atomicMin(&cmin[c], L.lo[e]);
            atomicMax(&cmax[c], L.hi[e]);
        }
    }
}

// One thread per (tile, ray, lane of the ray's group); wavefronts never
// straddle tiles (64 G threads per tile), hence never scenes.  One wavefront
// per workgroup, as in the single-volume raycast.
template <typename S, int G, bool kDense>
__global__ __launch_bounds__(64) void batch_raycast(const SceneDesc *__restrict__ sd, int n, uint32_t total_tiles)
{
    const long long gt = (long long)blockIdx.x * 64 + threadIdx.x;
    const uint32_t tile = (uint32_t)(gt / (64 * G));
    if (tile >= total_tiles) return;
    // 64 G consecutive threads share a tile, so the scene is wave-uniform
    const int s = __builtin_amdgcn_readfirstlane(scene_of(sd, n, tile, true));
    const SceneDesc &d = sd[s];
    if (!d.active) return;
    raycast_body<S, G, kDense>(d.v, d.cam, d.stamp, d.tiles_x8, d.tiles_y8, d.vertex, d.normal,
                               gt - (long long)d.ray_base * 64 * G);
}

// The whole step in one cooperative launch: the six phases above run one
// after the other inside a resident grid (the launch fails, and nothing runs,
// when the grid cannot be resident at once), separated by grid barriers.
// Every phase is the same body over the same work decomposition as its
// separate kernel, so the results are those of the six launches.  Every
// workgroup reaches every barrier: no phase returns early.
template <typename S, int G, bool kDense, bool kMlp>
__global__ __launch_bounds__(256) void batch_persistent(const SceneDesc *__restrict__ sd, int n, uint32_t prep_total,
                                                        uint32_t ray_total)
{
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    __shared__ uint32_t pre[kMaxScenes + 1];
    __shared__ SpanLds L;
    const int tid = threadIdx.x, lane = tid & 63;
    // frame reset
    for (uint32_t s = blockIdx.x; s < (uint32_t)n; s += gridDim.x)
        if (sd[s].active) frame_begin_body(sd[s].v.state, sd[s].v.ctr, tid);
    grid.sync();
    // pixel preparation: one 16x16 tile per workgroup and iteration
    for (uint32_t w = blockIdx.x; w < prep_total; w += gridDim.x) {
        const SceneDesc &d = sd[scene_of(sd, n, w, false)];
        if (d.active) {   // uniform over the workgroup
            const uint32_t local = w - d.prep_base;
            prep_body<kMlp>(d.v, d.depth, d.cam, d.noise, (int)(local % (uint32_t)d.tiles_x16),
                            (int)(local / (uint32_t)d.tiles_x16));
        }
        __syncthreads();   // the next tile reuses the preparation's LDS
    }
    grid.sync();
    // block fusion over every scene's candidates, one wavefront per candidate
    {
        scene_prefix<false>(sd, n, pre);
        const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * 4u + (tid >> 6));
        const uint32_t nwaves = gridDim.x * 4u;
        if (blockIdx.x == 0 && tid < n && sd[tid].active)
            atomicAdd(&sd[tid].v.state->total_candidates, (unsigned long long)(pre[tid + 1] - pre[tid]));
        FuseAcc acc;
        int cur = -1;
        for (uint32_t g = wave; g < pre[n]; g += nwaves) {
            const int s = scene_at(pre, n, g);
            if (s != cur) {
                if (cur >= 0) fuse_flush(sd[cur].v, acc, wave, lane);
                cur = s;
            }
            const SceneDesc &d = sd[s];
            fuse_block<S>(d.v, d.cam, d.fc, d.v.cand_list[g - pre[s]], lane, acc);
        }
        if (cur >= 0) fuse_flush(sd[cur].v, acc, wave, lane);
    }
    grid.sync();
    // span reset
    for (long long gt = (long long)blockIdx.x * 256 + tid; gt < (long long)ray_total * 64;
         gt += (long long)gridDim.x * 256) {
        const uint32_t tile = (uint32_t)(gt >> 6);
        const SceneDesc &d = sd[scene_of(sd, n, tile, true)];
        if (d.active)
            range_clear_body(d.v, d.tiles_x8, d.tiles_y8, d.cam.width, d.cam.height, gt - (long long)d.ray_base * 64);
    }
    grid.sync();
    // range pass over every scene's blocks
    {
        span_lds_init(L);
        scene_prefix<true>(sd, n, pre);   // (synchronises the workgroup)
        for (uint32_t g = blockIdx.x * 256u + tid; g < pre[n]; g += gridDim.x * 256u) {
            int s = 0;
            for (int k = 1; k < n; ++k) s += pre[k] <= g ? 1 : 0;
            const SceneDesc &d = sd[s];
            range_block(d.v, d.cam, d.stamp, d.tiles_x8, d.tiles_y8, g - pre[s],
                        [&](uint32_t c, uint32_t zl, uint32_t zh) {
                            if (!span_lds_add(L, ((uint32_t)s << 26) | c, zl, zh)) {
                                uint32_t *cmin = d.v.pix_range;
                                uint32_t *cmax = cmin + (size_t)((d.cam.width + kCell - 1) / kCell) *
                                                            ((d.cam.height + kCell - 1) / kCell);
                                atomicMin(&cmin[c], zl);
                                atomicMax(&cmax[c], zh);
                            }
                        });
        }
        __syncthreads();
        for (int e = tid; e < kSpanLds; e += 256) {
            const uint32_t key = L.key[e];
            if (key != kSpanEmpty) {
                const SceneDesc &d = sd[key >> 26];
                const uint32_t c = key & ((1u << 26) - 1u);
                uint32_t *cmin = d.v.pix_range;
                uint32_t *cmax =
                    cmin + (size_t)((d.cam.width + kCell - 1) / kCell) * ((d.cam.height + kCell - 1) / kCell);
                atomicMin(&cmin[c], L.lo[e]);
                atomicMax(&cmax[c], L.hi[e]);
            }
        }
    }
    grid.sync();
    // raycast: 256-thread chunks of the (tile, ray, lane) space; a wavefront's
    // 64 threads lie in one tile, so the tests below are wave-uniform
    const long long total = (long long)ray_total * 64 * G;
    for (long long base = (long long)blockIdx.x * 256; base < total; base += (long long)gridDim.x * 256) {
        const long long gt = base + tid;
        const uint32_t tile = (uint32_t)(gt / (64 * G));
        if (tile < ray_total) {
            const int s = __builtin_amdgcn_readfirstlane(scene_of(sd, n, tile, true));
            const SceneDesc &d = sd[s];
            if (d.active)
                raycast_body<S, G, kDense>(d.v, d.cam, d.stamp, d.tiles_x8, d.tiles_y8, d.vertex, d.normal,
                                           gt - (long long)d.ray_base * 64 * G);
        }
    }
}

}  // namespace tsdf

using namespace tsdf;

struct tsdf_batch {
    std::vector<tsdf_volume *> vols;
    std::vector<tsdf_intrinsics> K;
    SceneDesc *dev;
    std::vector<SceneDesc> host;
    uint32_t prep_total, ray_total;
    int32_t storage, dense, group;
    bool use_graph;
    bool persistent;     // one cooperative launch per step instead of six
    uint32_t fuse_grid;  // workgroups of the persistent fusion launch
    int32_t coop_grid;   // resident workgroups of the cooperative kernel last launched (0: not yet)
    const void *coop_fn;
    hipGraphExec_t exec;
    int32_t graph_key;   // (noise kind, group) the graph was captured for; -1 = none
};

static bool batch_intrinsics_ok(const tsdf_intrinsics *K)
{
    return K && isfinite(K->fx) && isfinite(K->fy) && isfinite(K->cx) && isfinite(K->cy) && K->fx > 0 &&
           K->fy > 0 && K->width > 0 && K->height > 0 && K->width <= 16384 && K->height <= 16384;
}

template <typename S, bool kDense>
static void launch_batch_raycast(int G, dim3 grid, hipStream_t s, const SceneDesc *sd, int n, uint32_t tiles)
{
    switch (G) {
    case 1: hipLaunchKernelGGL((batch_raycast<S, 1, kDense>), grid, dim3(64), 0, s, sd, n, tiles); break;
    case 2: hipLaunchKernelGGL((batch_raycast<S, 2, kDense>), grid, dim3(64), 0, s, sd, n, tiles); break;
    case 4: hipLaunchKernelGGL((batch_raycast<S, 4, kDense>), grid, dim3(64), 0, s, sd, n, tiles); break;
    case 16: hipLaunchKernelGGL((batch_raycast<S, 16, kDense>), grid, dim3(64), 0, s, sd, n, tiles); break;
    default: hipLaunchKernelGGL((batch_raycast<S, 8, kDense>), grid, dim3(64), 0, s, sd, n, tiles); break;
    }
}

static hipError_t enqueue_raycast(tsdf_batch *b, hipStream_t s)
{
    const int n = (int)b->vols.size();
    hipLaunchKernelGGL(batch_range_clear, dim3((unsigned)(((long long)b->ray_total * 64 + 255) / 256)), dim3(256), 0, s, b->dev, n,
                       b->ray_total);
    hipLaunchKernelGGL(batch_range, dim3(2048), dim3(256), 0, s, b->dev, n);
    const long long threads = (long long)b->ray_total * 64 * b->group;
    dim3 grid((unsigned)((threads + 63) / 64));
    if (b->storage == TSDF_F16) {
        if (b->dense) launch_batch_raycast<__half, true>(b->group, grid, s, b->dev, n, b->ray_total);
        else launch_batch_raycast<__half, false>(b->group, grid, s, b->dev, n, b->ray_total);
    } else {
        if (b->dense) launch_batch_raycast<float, true>(b->group, grid, s, b->dev, n, b->ray_total);
        else launch_batch_raycast<float, false>(b->group, grid, s, b->dev, n, b->ray_total);
    }
    return hipGetLastError();
}

// The step as one cooperative launch of batch_persistent, its grid the number
// of workgroups that can be resident at once (occupancy x CUs).
template <typename S, int G, bool kMlp>
static hipError_t launch_persistent_t(tsdf_batch *b, hipStream_t s)
{
    const void *fn = reinterpret_cast<const void *>(&batch_persistent<S, G, true, kMlp>);
    if (b->coop_fn != fn) {
        int per_cu = 0, dev = 0, cus = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, 0);
        if (e == hipSuccess) e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) return e;
        if (per_cu <= 0 || cus <= 0) return hipErrorInvalidConfiguration;
        b->coop_grid = per_cu * cus;
        b->coop_fn = fn;
    }
    const SceneDesc *sd = b->dev;
    int n = (int)b->vols.size();
    uint32_t pt = b->prep_total, rt = b->ray_total;
    void *args[] = {(void *)&sd, (void *)&n, (void *)&pt, (void *)&rt};
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)b->coop_grid), dim3(256), args, 0, s);
}

template <typename S, bool kMlp>
static hipError_t launch_persistent_g(tsdf_batch *b, hipStream_t s)
{
    switch (b->group) {
    case 1: return launch_persistent_t<S, 1, kMlp>(b, s);
    case 2: return launch_persistent_t<S, 2, kMlp>(b, s);
    case 4: return launch_persistent_t<S, 4, kMlp>(b, s);
    case 16: return launch_persistent_t<S, 16, kMlp>(b, s);
    default: return launch_persistent_t<S, 8, kMlp>(b, s);
    }
}

static hipError_t enqueue_persistent(tsdf_batch *b, int32_t noise_kind, hipStream_t s)
{
    const bool mlp = noise_kind == TSDF_NOISE_MLP;
    if (b->storage == TSDF_F16) return mlp ? launch_persistent_g<__half, true>(b, s) : launch_persistent_g<__half, false>(b, s);
    return mlp ? launch_persistent_g<float, true>(b, s) : launch_persistent_g<float, false>(b, s);
}

static hipError_t enqueue_step(tsdf_batch *b, int32_t noise_kind, hipStream_t s)
{
    const int n = (int)b->vols.size();
    hipLaunchKernelGGL(batch_frame_begin, dim3(n), dim3(kCtrLanes), 0, s, b->dev);
    if (noise_kind == TSDF_NOISE_MLP)
        hipLaunchKernelGGL(batch_prep<true>, dim3(b->prep_total), dim3(256), 0, s, b->dev, n);
    else
        hipLaunchKernelGGL(batch_prep<false>, dim3(b->prep_total), dim3(256), 0, s, b->dev, n);
    if (b->storage == TSDF_F16)
        hipLaunchKernelGGL(batch_fuse<__half>, dim3(b->fuse_grid), dim3(256), 0, s, b->dev, n);
    else
        hipLaunchKernelGGL(batch_fuse<float>, dim3(b->fuse_grid), dim3(256), 0, s, b->dev, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return enqueue_raycast(b, s);
}

static bool pose_ok(const double *p)
{
    for (int q = 0; q < 12; ++q)
        if (!isfinite(p[q])) return false;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            const double dot = p[4 * a] * p[4 * c] + p[4 * a + 1] * p[4 * c + 1] + p[4 * a + 2] * p[4 * c + 2];
            if (fabs(dot - (a == c ? 1.0 : 0.0)) > 1e-6) return false;
        }
    const double det = p[0] * (p[5] * p[10] - p[6] * p[9]) - p[1] * (p[4] * p[10] - p[6] * p[8]) +
                       p[2] * (p[4] * p[9] - p[5] * p[8]);
    return det > 0;
}

// Validates every scene's arguments, then fills the host table for this step
// and uploads it (stream-ordered after the previous step's kernels).  With
// depth_dev null every scene is active and only the raycast reads the table.
static tsdf_status stage_step(tsdf_batch *b, const float *const *depth_dev, const double *poses,
                              float *const *vertex_dev, float *const *normal_dev, const tsdf_noise_model *noise,
                              hipStream_t stream)
{
    const int n = (int)b->vols.size();
    for (int k = 0; k < n; ++k) {
        if (depth_dev && !depth_dev[k]) continue;
        if (!vertex_dev[k] || !normal_dev[k] || !pose_ok(poses + 12 * k)) return TSDF_EINVAL;
    }
    for (int k = 0; k < n; ++k) {
        SceneDesc &d = b->host[k];
        d.active = (!depth_dev || depth_dev[k]) ? 1u : 0u;
        if (!d.active) continue;
        tsdf_status st = volume_enqueue(b->vols[k], stream, &d.stamp);
        if (st != TSDF_OK) return st;
        const double *p = poses + 12 * k;
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c) d.cam.R[3 * r + c] = p[4 * r + c];
            d.cam.t[r] = p[4 * r + 3];
        }
        d.fc = make_fuse_cam(d.v, d.cam);
        d.depth = depth_dev ? depth_dev[k] : nullptr;
        d.vertex = (float4 *)vertex_dev[k];
        d.normal = (float4 *)normal_dev[k];
        d.noise.kind = noise ? noise->kind : TSDF_NOISE_QUADRATIC;
        d.noise.coeff = noise ? (float)noise->coeff : 0.0f;
        d.noise.mlp = noise ? noise->mlp_params_dev : nullptr;
    }
    // pageable source: the copy has read the table when the call returns
    hipError_t e = hipMemcpyAsync(b->dev, b->host.data(), sizeof(SceneDesc) * n, hipMemcpyHostToDevice, stream);
    return e == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

extern "C" {

uint64_t tsdf_batch_bytes(int32_t n_scenes)
{
    if (n_scenes <= 0 || n_scenes > kMaxScenes) return 0;
    return (sizeof(SceneDesc) * (uint64_t)n_scenes + 255) & ~255ull;
}

tsdf_status tsdf_batch_create(tsdf_volume *const *vols, const tsdf_intrinsics *K, int32_t n, void *dev_buf,
                              uint64_t bytes, tsdf_batch **out)
{
    if (!out) return TSDF_EINVAL;
    *out = nullptr;
    if (!vols || !K || n <= 0 || n > kMaxScenes || !dev_buf || bytes < tsdf_batch_bytes(n)) return TSDF_EINVAL;
    tsdf_batch *b = new (std::nothrow) tsdf_batch;
    if (!b) return TSDF_ENOMEM;
    b->dev = (SceneDesc *)dev_buf;
    b->host.assign(n, SceneDesc());
    b->prep_total = b->ray_total = 0;
    b->use_graph = false;
    b->persistent = false;
    b->fuse_grid = kFuseGrid;
    b->coop_grid = 0;
    b->coop_fn = nullptr;
    b->exec = nullptr;
    b->graph_key = -1;
    b->group = 8;
    for (int k = 0; k < n; ++k) {
        bool dup = false;
        for (int q = 0; q < k; ++q) dup |= vols[q] == vols[k];
        if (!vols[k] || dup || !batch_intrinsics_ok(&K[k])) {
            delete b;
            return TSDF_EINVAL;
        }
        const VolumeView v = volume_view(vols[k]);
        if (K[k].width > v.max_width || K[k].height > v.max_height) {
            delete b;
            return TSDF_EINVAL;
        }
        const int32_t dense = v.block_index != nullptr;
        if (k == 0) {
            b->storage = v.storage;
            b->dense = dense;
        } else if (v.storage != b->storage || dense != b->dense) {
            delete b;
            return TSDF_EINVAL;   // one storage type and index mode per batch
        }
        b->vols.push_back(vols[k]);
        b->K.push_back(K[k]);
        SceneDesc &d = b->host[k];
        memset(&d, 0, sizeof(d));
        d.v = v;
        d.cam.fx = K[k].fx;
        d.cam.fy = K[k].fy;
        d.cam.cx = K[k].cx;
        d.cam.cy = K[k].cy;
        d.cam.width = K[k].width;
        d.cam.height = K[k].height;
        d.tiles_x16 = (K[k].width + 15) / 16;
        d.tiles_y16 = (K[k].height + 15) / 16;
        d.tiles_x8 = (K[k].width + 7) / 8;
        d.tiles_y8 = (K[k].height + 7) / 8;
        d.prep_base = b->prep_total;
        d.ray_base = b->ray_total;
        b->prep_total += (uint32_t)(d.tiles_x16 * d.tiles_y16);
        b->ray_total += (uint32_t)(d.tiles_x8 * d.tiles_y8);
    }
    *out = b;
    return TSDF_OK;
}

void tsdf_batch_destroy(tsdf_batch *b)
{
    if (!b) return;
    if (b->exec) hipGraphExecDestroy(b->exec);
    delete b;
}

tsdf_status tsdf_batch_set_graph(tsdf_batch *b, int32_t enable)
{
    if (!b) return TSDF_EINVAL;
    b->use_graph = enable != 0;
    return TSDF_OK;
}

tsdf_status tsdf_batch_set_persistent(tsdf_batch *b, int32_t enable)
{
    if (!b || (enable && !b->dense)) return TSDF_EINVAL;
    b->persistent = enable != 0;
    return TSDF_OK;
}

tsdf_status tsdf_batch_set_raycast_group(tsdf_batch *b, int32_t group)
{
    if (!b || !(group == 1 || group == 2 || group == 4 || group == 8 || group == 16)) return TSDF_EINVAL;
    b->group = group;
    return TSDF_OK;
}

int32_t tsdf_batch_get_raycast_group(const tsdf_batch *b) { return b ? b->group : 0; }

tsdf_status tsdf_batch_step(tsdf_batch *b, const float *const *depth_dev, const double *poses_c2w,
                            float *const *vertex_dev, float *const *normal_dev, const tsdf_noise_model *noise,
                            hipStream_t stream)
{
    if (!b || !depth_dev || !poses_c2w || !vertex_dev || !normal_dev) return TSDF_EINVAL;
    const int32_t kind = noise ? noise->kind : TSDF_NOISE_QUADRATIC;
    if (kind != TSDF_NOISE_QUADRATIC && kind != TSDF_NOISE_CONSTANT && kind != TSDF_NOISE_MLP) return TSDF_EINVAL;
    if (kind == TSDF_NOISE_MLP && !noise->mlp_params_dev) return TSDF_EINVAL;
    if (noise && (!isfinite(noise->coeff) || noise->coeff < 0)) return TSDF_EINVAL;
    if (b->use_graph && !stream) return TSDF_EINVAL;   // capture needs a created stream
    tsdf_status st = stage_step(b, depth_dev, poses_c2w, vertex_dev, normal_dev, noise, stream);
    if (st != TSDF_OK) return st;
    if (b->persistent) return enqueue_persistent(b, kind, stream) == hipSuccess ? TSDF_OK : TSDF_EHIP;
    if (!b->use_graph) return enqueue_step(b, kind, stream) == hipSuccess ? TSDF_OK : TSDF_EHIP;
    const int32_t key = (kind * 64 + b->group) * 65536 + (int32_t)b->fuse_grid;
    if (!b->exec || b->graph_key != key) {
        if (b->exec) {
            hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return TSDF_EHIP;
        hipError_t e = enqueue_step(b, kind, stream);
        hipError_t e2 = hipStreamEndCapture(stream, &graph);
        if (e != hipSuccess || e2 != hipSuccess || !graph) {
            if (graph) hipGraphDestroy(graph);
            return TSDF_EHIP;
        }
        e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) {
            b->exec = nullptr;
            return TSDF_EHIP;
        }
        b->graph_key = key;
    }
    return hipGraphLaunch(b->exec, stream) == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

tsdf_status tsdf_batch_set_fuse_grid(tsdf_batch *b, uint32_t workgroups)
{
    if (!b || workgroups < 1 || workgroups > 65536) return TSDF_EINVAL;
    b->fuse_grid = workgroups;
    return TSDF_OK;
}

uint32_t tsdf_batch_get_fuse_grid(const tsdf_batch *b) { return b ? b->fuse_grid : 0; }

tsdf_status tsdf_batch_autotune_fuse(tsdf_batch *b, const float *const *depth_dev, const double *poses_c2w,
                                     float *const *vertex_dev, float *const *normal_dev,
                                     const tsdf_noise_model *noise, int32_t reps, hipStream_t stream,
                                     uint32_t *best_grid, float *best_ms)
{
    if (!b || !depth_dev || !poses_c2w || !vertex_dev || !normal_dev || reps < 1 || !best_grid || !best_ms)
        return TSDF_EINVAL;
    const int32_t kind = noise ? noise->kind : TSDF_NOISE_QUADRATIC;
    if (kind != TSDF_NOISE_QUADRATIC && kind != TSDF_NOISE_CONSTANT && kind != TSDF_NOISE_MLP) return TSDF_EINVAL;
    if (kind == TSDF_NOISE_MLP && !noise->mlp_params_dev) return TSDF_EINVAL;
    // persistent fusion grids of 1, 1.5, 2, 3 and 4 rounds of resident waves
    // (five per SIMD on 256 CUs: 1280 workgroups of four wavefronts a round)
    const uint32_t candidates[5] = {1280, 1920, 2560, 3840, 5120};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return TSDF_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return TSDF_EHIP;
    }
    tsdf_status st = TSDF_OK;
    float best = 3.4e38f;
    uint32_t bestg = b->fuse_grid;
    for (int c = 0; c < 5 && st == TSDF_OK; ++c) {
        b->fuse_grid = candidates[c];
        st = stage_step(b, depth_dev, poses_c2w, vertex_dev, normal_dev, noise, stream);
        if (st == TSDF_OK && enqueue_step(b, kind, stream) != hipSuccess) st = TSDF_EHIP;   // warm-up
        if (st == TSDF_OK && hipEventRecord(e0, stream) != hipSuccess) st = TSDF_EHIP;
        for (int r = 0; r < reps && st == TSDF_OK; ++r) {
            st = stage_step(b, depth_dev, poses_c2w, vertex_dev, normal_dev, noise, stream);
            if (st == TSDF_OK && enqueue_step(b, kind, stream) != hipSuccess) st = TSDF_EHIP;
        }
        float ms = 0.0f;
        if (st == TSDF_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = TSDF_EHIP;
        if (st == TSDF_OK && ms / reps < best) {
            best = ms / reps;
            bestg = candidates[c];
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    b->fuse_grid = bestg;
    *best_grid = bestg;
    *best_ms = best;
    return st;
}

tsdf_status tsdf_batch_autotune_raycast(tsdf_batch *b, const double *poses_c2w, float *const *vertex_dev,
                                        float *const *normal_dev, int32_t reps, hipStream_t stream,
                                        int32_t *best_group, float *best_ms)
{
    if (!b || !poses_c2w || !vertex_dev || !normal_dev || reps < 1 || !best_group || !best_ms) return TSDF_EINVAL;
    tsdf_status st = stage_step(b, nullptr, poses_c2w, vertex_dev, normal_dev, nullptr, stream);
    if (st != TSDF_OK) return st;
    const int candidates[5] = {1, 2, 4, 8, 16};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return TSDF_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return TSDF_EHIP;
    }
    float best = 3.4e38f;
    int bestg = b->group;
    for (int c = 0; c < 5 && st == TSDF_OK; ++c) {
        b->group = candidates[c];
        if (enqueue_raycast(b, stream) != hipSuccess) st = TSDF_EHIP;
        if (st == TSDF_OK && hipEventRecord(e0, stream) != hipSuccess) st = TSDF_EHIP;
        for (int r = 0; r < reps && st == TSDF_OK; ++r)
            if (enqueue_raycast(b, stream) != hipSuccess) st = TSDF_EHIP;
        float ms = 0.0f;
        if (st == TSDF_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = TSDF_EHIP;
        if (st == TSDF_OK && ms / reps < best) {
            best = ms / reps;
            bestg = candidates[c];
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    b->group = bestg;
    *best_group = bestg;
    *best_ms = best;
    return st;
}

}  // extern "C"

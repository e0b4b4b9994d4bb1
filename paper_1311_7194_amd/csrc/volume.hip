// Volume object, buffer layout, maintenance kernels and the C ABI of libtsdf.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <new>
#include <vector>

#include "tsdf_internal.h"

namespace tsdf {

// ------------------------------------------------------------ maintenance

__global__ void fill_u32_kernel(uint32_t *p, uint64_t n, uint32_t value)
{
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x)
        p[k] = value;
}

static hipError_t fill_u32(uint32_t *p, uint64_t n, uint32_t value, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

// keys of every hash entry, written at the entry's pool slot
__global__ void export_keys_kernel(VolumeView v, int32_t *keys, uint32_t cap)
{
    for (uint64_t h = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; h <= v.hash_mask;
         h += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long e = v.hash[h];
        if (e == kEmptyEntry) continue;
        const uint32_t slot = (uint32_t)(e >> 32);
        if (slot >= cap) continue;
        int bx, by, bz;
        unpack_key((uint32_t)(e & 0xffffffffu), bx, by, bz);
        keys[3 * (size_t)slot + 0] = bx;
        keys[3 * (size_t)slot + 1] = by;
        keys[3 * (size_t)slot + 2] = bz;
    }
}

hipError_t launch_export(const VolumeView &v, int32_t *keys, void *T, void *P, uint32_t cap, hipStream_t s)
{
    (void)T;
    (void)P;
    uint64_t slots = (uint64_t)v.hash_mask + 1;
    uint64_t blocks = (slots + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(export_keys_kernel, dim3((unsigned)blocks), dim3(256), 0, s, v, keys, cap);
    return hipGetLastError();
}

// one wavefront per imported block
template <typename S>
__global__ __launch_bounds__(256) void import_kernel(VolumeView v, const int32_t *keys, const S *T, const S *P,
                                                     uint32_t n)
{
    const int lane = threadIdx.x & 63;
    const uint32_t w = blockIdx.x * 4u + (threadIdx.x >> 6);
    if (w >= n) return;
    const int bx = keys[3 * (size_t)w], by = keys[3 * (size_t)w + 1], bz = keys[3 * (size_t)w + 2];
    if (bx < 0 || by < 0 || bz < 0 || bx >= v.nblk[0] || by >= v.nblk[1] || bz >= v.nblk[2]) {
        return;
    }
    const uint32_t key = pack_key(bx, by, bz);
    int32_t slot = -1;
    if (lane == 0) {
        slot = hash_find(v, key);
        if (slot < 0) {
            slot = hash_insert_unique(v, key);
            if (slot >= 0) {
                uint64_t b = block_linear(v, bx, by, bz);
                atomicOr(&v.occupancy[b >> 5], 1u << (b & 31));
            }
        }
    }
    slot = __shfl(slot, 0);
    if (slot < 0) return;
    S *dT = (S *)v.poolT + (size_t)slot * kBlockVoxels;
    S *dP = (S *)v.poolP + (size_t)slot * kBlockVoxels;
    uint32_t kmin = kKeyPosInf, zmask = 0;
    // lane = x + 8 y holds the column of voxels lane + 64 z
    for (int k = lane; k < kBlockVoxels; k += 64) {
        const S t = T[(size_t)w * kBlockVoxels + k];
        dT[k] = t;
        dP[k] = P[(size_t)w * kBlockVoxels + k];
        const float f = (float)t;
        if (fabsf(f) <= 1.0f) {
            kmin = min(kmin, order_key(f));
            zmask |= 1u << (k >> 6);
        }
    }
    kmin = wave_min_u32(kmin);
    const uint32_t box = wave_box(zmask);
    if (lane == 0) {
        v.block_min[slot] = kmin;
        v.block_box[slot] = box;
        if (v.block_index) v.block_index[block_linear(v, bx, by, bz)] = slot | (kmin > kKeyZero ? kIndexPositive : 0);
    }
}

hipError_t launch_import(const VolumeView &v, const int32_t *keys, const void *T, const void *P, uint32_t n,
                         hipStream_t s)
{
    if (n == 0) return hipSuccess;
    dim3 grid((n + 3) / 4);
    if (v.storage == TSDF_F16)
        hipLaunchKernelGGL(import_kernel<__half>, grid, dim3(256), 0, s, v, keys, (const __half *)T,
                           (const __half *)P, n);
    else
        hipLaunchKernelGGL(import_kernel<float>, grid, dim3(256), 0, s, v, keys, (const float *)T,
                           (const float *)P, n);
    return hipGetLastError();
}

// ------------------------------------------------------------ layout

struct Layout {
    uint64_t state, ctr, hash, occupancy, block_index, cand_bits, cand_list, pixmap, pool_keys, block_min, block_box, tile_range, pix_range, mark_bits,
        poolT, poolP, total;
    uint64_t bitmap_words, tile_words, nblocks;
};

static uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

static bool valid_desc(const tsdf_volume_desc *d)
{
    if (!d) return false;
    for (int a = 0; a < 3; ++a)
        if (d->dims[a] <= 0 || d->dims[a] % kBlock != 0 || d->dims[a] > 8192) return false;
    if (!(d->voxel_size > 0) || !isfinite(d->voxel_size)) return false;
    for (int a = 0; a < 3; ++a)
        if (!isfinite(d->origin[a])) return false;
    if (!(d->trunc_voxels > 0) || !isfinite(d->trunc_voxels)) return false;
    if (d->capacity_blocks == 0 || d->capacity_blocks > kMaxCapacity) return false;
    if (d->hash_slots == 0 || (d->hash_slots & (d->hash_slots - 1)) != 0) return false;
    if ((uint64_t)d->hash_slots < 2ull * d->capacity_blocks) return false;
    if (d->storage != TSDF_F32 && d->storage != TSDF_F16) return false;
    if (!(d->q_hat >= 0) || !isfinite(d->q_hat)) return false;
    if (d->max_width <= 0 || d->max_height <= 0 || d->max_width > 16384 || d->max_height > 16384) return false;
    if (d->dense_index != 0 && d->dense_index != 1) return false;
    return true;
}

static Layout layout_of(const tsdf_volume_desc *d)
{
    Layout L;
    uint64_t nblocks = 1;
    for (int a = 0; a < 3; ++a) nblocks *= (uint64_t)(d->dims[a] / kBlock);
    L.bitmap_words = (nblocks + 31) / 32;
    L.nblocks = nblocks;
    uint32_t maxc = d->max_candidates ? d->max_candidates : d->capacity_blocks;
    uint64_t elem = d->storage == TSDF_F16 ? 2 : 4;
    uint64_t off = 0;
    L.state = off;
    off = align256(off + sizeof(DeviceState));
    L.ctr = off;
    off = align256(off + sizeof(Counters));
    L.hash = off;
    off = align256(off + 8ull * d->hash_slots);
    L.occupancy = off;
    off = align256(off + 4ull * L.bitmap_words);
    L.block_index = off;
    if (d->dense_index) off = align256(off + 4ull * nblocks);
    L.cand_bits = off;
    off = align256(off + 4ull * L.bitmap_words);
    L.mark_bits = off;
    off = align256(off + 4ull * L.bitmap_words);
    L.cand_list = off;
    off = align256(off + 4ull * maxc);
    L.pixmap = off;
    off = align256(off + 8ull * (uint64_t)d->max_width * (uint64_t)d->max_height);
    L.pool_keys = off;
    off = align256(off + 4ull * d->capacity_blocks);
    L.block_min = off;
    off = align256(off + 4ull * d->capacity_blocks);
    L.block_box = off;
    off = align256(off + 4ull * d->capacity_blocks);
    L.tile_words = (uint64_t)((d->max_width + 7) / 8) * (uint64_t)((d->max_height + 7) / 8);
    L.tile_range = off;
    off = align256(off + 8ull * L.tile_words);
    L.pix_range = off;
    off = align256(off + 8ull * (uint64_t)((d->max_width + kCell - 1) / kCell) *
                             (uint64_t)((d->max_height + kCell - 1) / kCell));
    // one block past the capacity: the chi block that absent neighbours read
    L.poolT = off;
    off = align256(off + elem * kBlockVoxels * ((uint64_t)d->capacity_blocks + 1));
    L.poolP = off;
    off = align256(off + elem * kBlockVoxels * ((uint64_t)d->capacity_blocks + 1));
    L.total = off;
    return L;
}

}  // namespace tsdf

using namespace tsdf;

enum { STAGE_PREP = 0, STAGE_FUSE = 1, STAGE_RANGE = 2, STAGE_RAYCAST = 3, N_STAGES = 4 };

struct EventPair {
    int stage;
    hipEvent_t start, stop;
};

struct tsdf_volume {
    tsdf_volume_desc desc;
    Layout layout;
    VolumeView view;
    uint8_t *base;
    hipStream_t last_stream;
    uint32_t host_flags;   // sticky flags seen by the last tsdf_query_stats
    uint32_t raycast_stamp;
    int32_t ray_group;     // lanes per ray in the raycast march (1, 2, 4, 8 or 16)
    bool timing;
    std::vector<EventPair> pending;   // recorded, not yet read
    std::vector<hipEvent_t> spare;    // events ready for reuse
    double stage_ms[N_STAGES];
    uint64_t stage_launches[N_STAGES];
};

namespace tsdf {

VolumeView volume_view(const tsdf_volume *vol) { return vol->view; }

tsdf_status volume_enqueue(tsdf_volume *vol, hipStream_t s, uint32_t *stamp)
{
    if (vol->host_flags) return TSDF_EFULL;
    vol->last_stream = s;
    if (stamp) *stamp = ++vol->raycast_stamp == 0 ? ++vol->raycast_stamp : vol->raycast_stamp;
    return TSDF_OK;
}

void volume_note_flags(tsdf_volume *vol, uint32_t flags) { vol->host_flags |= flags; }

}  // namespace tsdf

static hipEvent_t take_event(tsdf_volume *v)
{
    if (!v->spare.empty()) {
        hipEvent_t e = v->spare.back();
        v->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch `fn` bracketed by timing events when timing is on.
template <typename F>
static hipError_t timed(tsdf_volume *v, int stage, hipStream_t s, F fn)
{
    if (!v->timing) return fn();
    EventPair p{stage, take_event(v), take_event(v)};
    if (!p.start || !p.stop) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(p.start, s);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(p.stop, s);
    v->pending.push_back(p);
    return e;
}

static hipError_t collect_timing(tsdf_volume *v)
{
    hipError_t err = hipSuccess;
    for (EventPair &p : v->pending) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(p.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.start, p.stop);
        if (e == hipSuccess) {
            v->stage_ms[p.stage] += ms;
            v->stage_launches[p.stage] += 1;
        } else {
            err = e;
        }
        v->spare.push_back(p.start);
        v->spare.push_back(p.stop);
    }
    v->pending.clear();
    return err;
}

static bool valid_pose(const double *p)
{
    if (!p) return false;
    for (int k = 0; k < 12; ++k)
        if (!isfinite(p[k])) return false;
    // rows of R must be orthonormal and det(R) = +1 (tolerance 1e-6)
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double dot = p[4 * a] * p[4 * b] + p[4 * a + 1] * p[4 * b + 1] + p[4 * a + 2] * p[4 * b + 2];
            if (fabs(dot - (a == b ? 1.0 : 0.0)) > 1e-6) return false;
        }
    double det = p[0] * (p[5] * p[10] - p[6] * p[9]) - p[1] * (p[4] * p[10] - p[6] * p[8]) +
                 p[2] * (p[4] * p[9] - p[5] * p[8]);
    return det > 0;
}

static bool valid_intrinsics(const tsdf_intrinsics *K)
{
    return K && isfinite(K->fx) && isfinite(K->fy) && isfinite(K->cx) && isfinite(K->cy) && K->fx > 0 &&
           K->fy > 0 && K->width > 0 && K->height > 0 && K->width <= 16384 && K->height <= 16384;
}

static Camera make_camera(const tsdf_intrinsics *K, const double *pose)
{
    Camera c;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) c.R[3 * r + k] = pose[4 * r + k];
        c.t[r] = pose[4 * r + 3];
    }
    c.fx = K->fx;
    c.fy = K->fy;
    c.cx = K->cx;
    c.cy = K->cy;
    c.width = K->width;
    c.height = K->height;
    return c;
}

static tsdf_status hip_status(hipError_t e) { return e == hipSuccess ? TSDF_OK : TSDF_EHIP; }

static tsdf_status clear_volume(tsdf_volume *v, hipStream_t s)
{
    const Layout &L = v->layout;
    hipError_t e = fill_u32((uint32_t *)(v->base + L.state), sizeof(DeviceState) / 4, 0u, s);
    if (e == hipSuccess) e = fill_u32((uint32_t *)(v->base + L.ctr), sizeof(Counters) / 4, 0u, s);
    // tile ranges: [0, n) min depths (+inf), [n, 2n) max depths (0)
    if (e == hipSuccess) e = fill_u32((uint32_t *)(v->base + L.tile_range), L.tile_words, 0x7f800000u, s);
    if (e == hipSuccess) e = fill_u32((uint32_t *)(v->base + L.tile_range) + L.tile_words, L.tile_words, 0u, s);
    if (e == hipSuccess) e = fill_u32((uint32_t *)(v->base + L.hash), 2ull * v->desc.hash_slots, 0xffffffffu, s);
    if (e == hipSuccess) e = fill_u32((uint32_t *)(v->base + L.occupancy), L.bitmap_words, 0u, s);
    if (e == hipSuccess && v->desc.dense_index)
        e = fill_u32((uint32_t *)(v->base + L.block_index), L.nblocks, 0xffffffffu, s);
    if (e == hipSuccess) e = fill_u32((uint32_t *)(v->base + L.cand_bits), L.bitmap_words, 0u, s);
    // the chi block (T = 2 in either storage type, P = 0)
    const uint64_t elem = v->desc.storage == TSDF_F16 ? 2 : 4;
    const uint64_t chi_off = elem * kBlockVoxels * (uint64_t)v->desc.capacity_blocks;
    const uint32_t chi_word = v->desc.storage == TSDF_F16 ? 0x40004000u : 0x40000000u;
    if (e == hipSuccess) e = fill_u32((uint32_t *)(v->base + L.poolT + chi_off), elem * kBlockVoxels / 4, chi_word, s);
    if (e == hipSuccess) e = fill_u32((uint32_t *)(v->base + L.poolP + chi_off), elem * kBlockVoxels / 4, 0u, s);
    v->host_flags = 0;
    v->last_stream = s;
    return hip_status(e);
}

extern "C" {

const char *tsdf_status_string(tsdf_status s)
{
    switch (s) {
    case TSDF_OK: return "ok";
    case TSDF_EINVAL: return "invalid argument";
    case TSDF_ENOMEM: return "buffer too small";
    case TSDF_EFULL: return "block pool, hash table or candidate list exhausted";
    case TSDF_EHIP: return "HIP runtime error";
    case TSDF_ESTATE: return "invalid state";
    }
    return "unknown status";
}

tsdf_status tsdf_volume_bytes(const tsdf_volume_desc *desc, uint64_t *bytes)
{
    if (!valid_desc(desc) || !bytes) return TSDF_EINVAL;
    *bytes = layout_of(desc).total;
    return TSDF_OK;
}

tsdf_status tsdf_create_volume(const tsdf_volume_desc *desc, void *dev_buf, uint64_t bytes, hipStream_t stream,
                               tsdf_volume **out)
{
    if (!out) return TSDF_EINVAL;
    *out = nullptr;
    if (!valid_desc(desc) || !dev_buf || ((uintptr_t)dev_buf & 255) != 0) return TSDF_EINVAL;
    Layout L = layout_of(desc);
    if (bytes < L.total) return TSDF_ENOMEM;
    tsdf_volume *v = new (std::nothrow) tsdf_volume;
    if (!v) return TSDF_ENOMEM;
    v->desc = *desc;
    if (v->desc.max_candidates == 0) v->desc.max_candidates = desc->capacity_blocks;
    v->layout = L;
    v->base = (uint8_t *)dev_buf;
    v->timing = false;
    for (int k = 0; k < N_STAGES; ++k) {
        v->stage_ms[k] = 0.0;
        v->stage_launches[k] = 0;
    }
    VolumeView &w = v->view;
    w.state = (DeviceState *)(v->base + L.state);
    w.ctr = (Counters *)(v->base + L.ctr);
    w.pool_keys = (uint32_t *)(v->base + L.pool_keys);
    w.block_min = (uint32_t *)(v->base + L.block_min);
    w.tile_range = (uint32_t *)(v->base + L.tile_range);
    w.pix_range = (uint32_t *)(v->base + L.pix_range);
    w.block_box = (uint32_t *)(v->base + L.block_box);
    w.mark_bits = (uint32_t *)(v->base + L.mark_bits);
    w.max_width = desc->max_width;
    w.max_height = desc->max_height;
    v->raycast_stamp = 0;
    v->ray_group = 8;
    w.hash = (unsigned long long *)(v->base + L.hash);
    w.occupancy = (uint32_t *)(v->base + L.occupancy);
    w.block_index = desc->dense_index ? (int32_t *)(v->base + L.block_index) : nullptr;
    w.cand_bits = (uint32_t *)(v->base + L.cand_bits);
    w.cand_list = (uint32_t *)(v->base + L.cand_list);
    w.pixmap = (float2 *)(v->base + L.pixmap);
    w.poolT = v->base + L.poolT;
    w.poolP = v->base + L.poolP;
    for (int a = 0; a < 3; ++a) {
        w.dims[a] = desc->dims[a];
        w.nblk[a] = desc->dims[a] / kBlock;
        w.origin[a] = desc->origin[a];
    }
    w.vs = desc->voxel_size;
    w.inv_vs = 1.0 / desc->voxel_size;
    w.delta = desc->trunc_voxels * desc->voxel_size;
    w.inv_delta = 1.0 / w.delta;
    w.q_hat = (float)desc->q_hat;
    w.rule = TSDF_RULE_KALMAN;
    w.weight_kind = TSDF_WEIGHT_CONSTANT;
    w.w = 1.0f;
    w.w_max = INFINITY;
    w.capacity = desc->capacity_blocks;
    w.hash_mask = desc->hash_slots - 1;
    w.max_candidates = v->desc.max_candidates;
    w.storage = desc->storage;
    tsdf_status st = clear_volume(v, stream);
    if (st != TSDF_OK) {
        delete v;
        return st;
    }
    *out = v;
    return TSDF_OK;
}

void tsdf_destroy_volume(tsdf_volume *vol)
{
    if (!vol) return;
    for (EventPair &p : vol->pending) {
        hipEventDestroy(p.start);
        hipEventDestroy(p.stop);
    }
    for (hipEvent_t e : vol->spare) hipEventDestroy(e);
    delete vol;
}

tsdf_status tsdf_set_update_rule(tsdf_volume *vol, int32_t rule, int32_t weight_kind, double w, double w_max)
{
    if (!vol) return TSDF_EINVAL;
    if (rule != TSDF_RULE_KALMAN && rule != TSDF_RULE_RUNNING && rule != TSDF_RULE_WEIGHTED) return TSDF_EINVAL;
    if (weight_kind != TSDF_WEIGHT_CONSTANT && weight_kind != TSDF_WEIGHT_INV_VARIANCE) return TSDF_EINVAL;
    if (rule == TSDF_RULE_RUNNING && (weight_kind != TSDF_WEIGHT_CONSTANT || !(w > 0.0 && w <= 1.0)))
        return TSDF_EINVAL;
    if (rule == TSDF_RULE_WEIGHTED) {
        if (weight_kind == TSDF_WEIGHT_CONSTANT && !(w > 0.0 && w <= 3.0e38)) return TSDF_EINVAL;
        if (!(w_max > 0.0)) return TSDF_EINVAL;
        if (vol->desc.storage == TSDF_F16 && !(w_max <= 65504.0)) return TSDF_EINVAL;
    }
    vol->view.rule = rule;
    vol->view.weight_kind = weight_kind;
    vol->view.w = (float)w;
    vol->view.w_max = (float)fmin(w_max, 3.0e38);
    if (isinf(w_max)) vol->view.w_max = INFINITY;
    return TSDF_OK;
}

tsdf_status tsdf_reset_volume(tsdf_volume *vol, hipStream_t stream)
{
    if (!vol) return TSDF_EINVAL;
    return clear_volume(vol, stream);
}

tsdf_status tsdf_integrate_frame(tsdf_volume *vol, const float *depth_dev, const tsdf_intrinsics *K,
                                 const double pose_c2w[12], const tsdf_noise_model *noise, hipStream_t stream)
{
    if (!vol || !depth_dev || !valid_intrinsics(K) || !valid_pose(pose_c2w) || !noise) return TSDF_EINVAL;
    if (K->width > vol->desc.max_width || K->height > vol->desc.max_height) return TSDF_EINVAL;
    if (!isfinite(noise->coeff) || noise->coeff < 0) return TSDF_EINVAL;
    if (noise->kind != TSDF_NOISE_QUADRATIC && noise->kind != TSDF_NOISE_CONSTANT && noise->kind != TSDF_NOISE_MLP)
        return TSDF_EINVAL;
    if (noise->kind == TSDF_NOISE_MLP && !noise->mlp_params_dev) return TSDF_EINVAL;
    if (vol->host_flags) return TSDF_EFULL;
    Camera cam = make_camera(K, pose_c2w);
    NoiseParams np;
    np.kind = noise->kind;
    np.coeff = (float)noise->coeff;
    np.mlp = noise->mlp_params_dev;
    vol->last_stream = stream;
    const VolumeView &w = vol->view;
    hipError_t e = launch_frame_begin(w, stream);
    if (e == hipSuccess)
        e = timed(vol, STAGE_PREP, stream, [&] { return launch_prep(w, depth_dev, cam, np, stream); });
    if (e == hipSuccess) e = timed(vol, STAGE_FUSE, stream, [&] { return launch_fuse(w, cam, stream); });
    return hip_status(e);
}

tsdf_status tsdf_raycast(tsdf_volume *vol, const tsdf_intrinsics *K, const double pose_c2w[12], float *vertex_dev,
                         float *normal_dev, hipStream_t stream)
{
    if (!vol || !valid_intrinsics(K) || !valid_pose(pose_c2w) || !vertex_dev || !normal_dev) return TSDF_EINVAL;
    if (K->width > vol->desc.max_width || K->height > vol->desc.max_height) return TSDF_EINVAL;
    Camera cam = make_camera(K, pose_c2w);
    vol->last_stream = stream;
    const VolumeView &w = vol->view;
    const uint32_t stamp = ++vol->raycast_stamp == 0 ? ++vol->raycast_stamp : vol->raycast_stamp;
    hipError_t e = timed(vol, STAGE_RANGE, stream, [&] { return launch_range(w, cam, stamp, stream); });
    if (e == hipSuccess)
        e = timed(vol, STAGE_RAYCAST, stream, [&] {
            return launch_march(w, cam, stamp, vol->ray_group, (float4 *)vertex_dev, (float4 *)normal_dev, stream);
        });
    return hip_status(e);
}

tsdf_status tsdf_raycast_footprint(tsdf_volume *vol, const tsdf_intrinsics *K, const double pose_c2w[12],
                                   float *vertex_dev, float *normal_dev, uint64_t *blocks_out, hipStream_t stream)
{
    if (!vol || !valid_intrinsics(K) || !valid_pose(pose_c2w) || !vertex_dev || !normal_dev || !blocks_out)
        return TSDF_EINVAL;
    if (K->width > vol->desc.max_width || K->height > vol->desc.max_height) return TSDF_EINVAL;
    Camera cam = make_camera(K, pose_c2w);
    vol->last_stream = stream;
    const VolumeView &w = vol->view;
    const uint32_t stamp = ++vol->raycast_stamp == 0 ? ++vol->raycast_stamp : vol->raycast_stamp;
    unsigned long long *count = &w.state->footprint;
    hipError_t e = fill_u32(w.mark_bits, vol->layout.bitmap_words, 0u, stream);
    if (e == hipSuccess) e = fill_u32((uint32_t *)count, 2, 0u, stream);
    if (e == hipSuccess) e = launch_range(w, cam, stamp, stream);
    if (e == hipSuccess)
        e = launch_march(w, cam, stamp, vol->ray_group, (float4 *)vertex_dev, (float4 *)normal_dev, stream, true);
    if (e == hipSuccess) e = launch_count_bits(w.mark_bits, vol->layout.bitmap_words, count, stream);
    unsigned long long host = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&host, count, sizeof(host), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return TSDF_EHIP;
    *blocks_out = host;
    return TSDF_OK;
}

tsdf_status tsdf_query_stats(tsdf_volume *vol, tsdf_stats *out)
{
    if (!vol || !out) return TSDF_EINVAL;
    DeviceState st;
    Counters *ctr = new (std::nothrow) Counters;
    if (!ctr) return TSDF_ENOMEM;
    hipError_t e = hipMemcpyAsync(&st, vol->view.state, sizeof(st), hipMemcpyDeviceToHost, vol->last_stream);
    if (e == hipSuccess) e = hipMemcpyAsync(ctr, vol->view.ctr, sizeof(Counters), hipMemcpyDeviceToHost, vol->last_stream);
    if (e == hipSuccess) e = hipStreamSynchronize(vol->last_stream);
    if (e != hipSuccess) {
        delete ctr;
        return TSDF_EHIP;
    }
    uint64_t fr[CTR_N] = {0, 0, 0, 0}, tot[CTR_N] = {0, 0, 0, 0};
    for (int l = 0; l < kCtrLanes; ++l)
        for (int c = 0; c < CTR_N; ++c) {
            fr[c] += ctr->frame[l][c];
            tot[c] += ctr->total[l][c];
        }
    delete ctr;
    out->allocated_blocks = st.pool_count < vol->desc.capacity_blocks ? st.pool_count : vol->desc.capacity_blocks;
    out->frame_candidates = st.cand_count;
    out->frame_new_blocks = fr[CTR_NEW];
    out->frame_updates = fr[CTR_UPDATES];
    out->frame_fresh_updates = fr[CTR_FRESH];
    out->total_updates = tot[CTR_UPDATES];
    out->total_fresh_updates = tot[CTR_FRESH];
    out->total_candidates = st.total_candidates;
    out->total_new_blocks = tot[CTR_NEW];
    out->frames = st.frames;
    out->frame_touched_blocks = fr[CTR_TOUCHED];
    out->total_touched_blocks = tot[CTR_TOUCHED];
    out->status_flags = st.status;
    out->reserved = 0;
    vol->host_flags = st.status;
    return TSDF_OK;
}

tsdf_status tsdf_set_raycast_group(tsdf_volume *vol, int32_t group)
{
    if (!vol || !(group == 1 || group == 2 || group == 4 || group == 8 || group == 16)) return TSDF_EINVAL;
    vol->ray_group = group;
    return TSDF_OK;
}

int32_t tsdf_get_raycast_group(const tsdf_volume *vol) { return vol ? vol->ray_group : 0; }

tsdf_status tsdf_autotune_raycast(tsdf_volume *vol, const tsdf_intrinsics *K, const double pose_c2w[12],
                                  float *vertex_dev, float *normal_dev, int32_t reps, hipStream_t stream,
                                  int32_t *best_group, float *best_ms)
{
    if (!vol || !valid_intrinsics(K) || !valid_pose(pose_c2w) || !vertex_dev || !normal_dev || reps < 1 ||
        !best_group || !best_ms)
        return TSDF_EINVAL;
    if (K->width > vol->desc.max_width || K->height > vol->desc.max_height) return TSDF_EINVAL;
    const int candidates[5] = {1, 2, 4, 8, 16};
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return TSDF_EHIP;
    const bool was_timing = vol->timing;
    vol->timing = false;
    float best = 3.4e38f;
    int bestg = vol->ray_group;
    tsdf_status st = TSDF_OK;
    for (int c = 0; c < 5 && st == TSDF_OK; ++c) {
        vol->ray_group = candidates[c];
        st = tsdf_raycast(vol, K, pose_c2w, vertex_dev, normal_dev, stream);   // warm-up
        if (st != TSDF_OK) break;
        if (hipEventRecord(e0, stream) != hipSuccess) st = TSDF_EHIP;
        for (int r = 0; r < reps && st == TSDF_OK; ++r) st = tsdf_raycast(vol, K, pose_c2w, vertex_dev, normal_dev, stream);
        if (st == TSDF_OK && hipEventRecord(e1, stream) != hipSuccess) st = TSDF_EHIP;
        float ms = 0.0f;
        if (st == TSDF_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = TSDF_EHIP;
        if (st == TSDF_OK && ms / reps < best) {
            best = ms / reps;
            bestg = candidates[c];
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    vol->timing = was_timing;
    vol->ray_group = bestg;
    *best_group = bestg;
    *best_ms = best;
    return st;
}

tsdf_status tsdf_set_timing(tsdf_volume *vol, int32_t enable)
{
    if (!vol) return TSDF_EINVAL;
    vol->timing = enable != 0;
    return TSDF_OK;
}

tsdf_status tsdf_read_timing(tsdf_volume *vol, tsdf_timing *out, int32_t reset)
{
    if (!vol || !out) return TSDF_EINVAL;
    hipError_t e = collect_timing(vol);
    out->prep_ms = vol->stage_ms[STAGE_PREP];
    out->fuse_ms = vol->stage_ms[STAGE_FUSE];
    out->range_ms = vol->stage_ms[STAGE_RANGE];
    out->raycast_ms = vol->stage_ms[STAGE_RAYCAST];
    out->prep_launches = vol->stage_launches[STAGE_PREP];
    out->fuse_launches = vol->stage_launches[STAGE_FUSE];
    out->range_launches = vol->stage_launches[STAGE_RANGE];
    out->raycast_launches = vol->stage_launches[STAGE_RAYCAST];
    if (reset)
        for (int k = 0; k < N_STAGES; ++k) {
            vol->stage_ms[k] = 0.0;
            vol->stage_launches[k] = 0;
        }
    return hip_status(e);
}

tsdf_status tsdf_export_blocks(tsdf_volume *vol, int32_t *keys_dev, void *T_dev, void *P_dev, uint64_t cap,
                               uint64_t *n_out, hipStream_t stream)
{
    if (!vol || !n_out || (cap > 0 && (!keys_dev || !T_dev || !P_dev))) return TSDF_EINVAL;
    DeviceState st;
    hipError_t e = hipMemcpyAsync(&st, vol->view.state, sizeof(st), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return TSDF_EHIP;
    uint64_t n = st.pool_count < vol->desc.capacity_blocks ? st.pool_count : vol->desc.capacity_blocks;
    *n_out = n;
    uint64_t m = n < cap ? n : cap;
    if (m == 0) return TSDF_OK;
    uint64_t elem = vol->desc.storage == TSDF_F16 ? 2 : 4;
    e = fill_u32((uint32_t *)keys_dev, 3 * m, 0xffffffffu, stream);
    if (e == hipSuccess) e = launch_export(vol->view, keys_dev, T_dev, P_dev, (uint32_t)m, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(T_dev, vol->view.poolT, m * kBlockVoxels * elem, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(P_dev, vol->view.poolP, m * kBlockVoxels * elem, hipMemcpyDeviceToDevice, stream);
    vol->last_stream = stream;
    return hip_status(e);
}

tsdf_status tsdf_import_blocks(tsdf_volume *vol, const int32_t *keys_dev, const void *T_dev, const void *P_dev,
                               uint64_t n, hipStream_t stream)
{
    if (!vol || (n > 0 && (!keys_dev || !T_dev || !P_dev)) || n > vol->desc.capacity_blocks) return TSDF_EINVAL;
    vol->last_stream = stream;
    return hip_status(launch_import(vol->view, keys_dev, T_dev, P_dev, (uint32_t)n, stream));
}

}  // extern "C"

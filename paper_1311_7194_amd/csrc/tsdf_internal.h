// Internal layout and kernel interfaces of libtsdf (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>
#include <string.h>

#include "tsdf.h"

namespace tsdf {

constexpr int kBlock = 8;              // voxels per block edge (M)
constexpr int kBlockVoxels = 512;      // M^3
constexpr float kChi = 2.0f;           // stored sentinel; any |T_hat| > 1 is chi
constexpr uint32_t kEmptyKey = 0xffffffffu;
constexpr uint64_t kEmptyEntry = ~0ull;
constexpr int kMaxProbes = 512;        // hash probe limit before HASH_FULL

// Device-resident state and sticky status (one 256-byte line).
struct DeviceState {
    uint32_t pool_count;     // blocks handed out (may exceed capacity after overflow)
    uint32_t status;         // TSDF_FLAG_* bits, sticky
    uint32_t cand_count;     // unique candidate blocks of the current frame
    uint32_t near_stamp;     // raycast call id whose range pass met a block at the camera plane
    unsigned long long frames;
    unsigned long long total_candidates;
    unsigned long long footprint;   // blocks counted by the last raycast footprint query
    uint32_t pad[54];
};
static_assert(sizeof(DeviceState) == 256, "state line");

// Event counters, spread over kCtrLanes addresses so that thousands of
// wavefronts do not serialise on one atomic; the host sums the lanes.
// Edge in pixels of the cells of the raycast's per-cell depth spans.
constexpr int kCell = 4;

constexpr int kCtrLanes = 256;
enum { CTR_UPDATES = 0, CTR_FRESH = 1, CTR_NEW = 2, CTR_TOUCHED = 3, CTR_N = 4 };
struct Counters {
    unsigned long long frame[kCtrLanes][CTR_N];
    unsigned long long total[kCtrLanes][CTR_N];
};

// Pointers into the caller's device buffer.
struct VolumeView {
    DeviceState *state;
    Counters *ctr;
    unsigned long long *hash;   // hash_slots entries: (slot << 32) | key, ~0 = empty
    uint32_t *pool_keys;        // capacity entries: key of the block in each pool slot
    uint32_t *block_min;        // capacity entries: ordered key of a lower bound of the block's non-chi T
    uint32_t *block_box;        // capacity entries: bounding box of the block's non-chi voxels (see box_*)
    uint32_t *tile_range;       // raycast: per 8x8 pixel tile (min depth bits, max depth bits)
    uint32_t *pix_range;        // raycast: per kCell x kCell pixel cell (min depth bits, max depth bits)
    uint32_t *mark_bits;        // one bit per virtual block: blocks a footprint query's rays read
    uint32_t *occupancy;        // one bit per block of the virtual grid
    int32_t *block_index;       // optional dense index per virtual block: slot | positive << 30, -1 = empty
    uint32_t *cand_bits;        // per-frame candidate dedup bits (all clear between frames)
    uint32_t *cand_list;        // max_candidates keys
    float2 *pixmap;             // per pixel (depth or 0, measurement variance p_hat)
    void *poolT;                // capacity * 512 * elem
    void *poolP;
    int32_t dims[3];
    int32_t nblk[3];
    double vs, inv_vs;
    double origin[3];
    double delta, inv_delta;
    float q_hat;
    int32_t rule;               // tsdf_update_rule
    int32_t weight_kind;        // tsdf_weight_kind
    float w, w_max;             // Algorithms 1 and 2: constant weight, cap of the weight sum
    uint32_t capacity;
    uint32_t hash_mask;
    uint32_t max_candidates;
    int32_t storage;            // TSDF_F32 / TSDF_F16
    int32_t max_width, max_height;
};

struct Camera {
    double R[9];      // row-major camera-to-world rotation
    double t[3];
    double fx, fy, cx, cy;
    int32_t width, height;
};

struct NoiseParams {
    int32_t kind;
    float coeff;
    const void *mlp;
};

// Block key: 10 bits per axis.
__host__ __device__ inline uint32_t pack_key(int bx, int by, int bz)
{
    return (uint32_t)bx | ((uint32_t)by << 10) | ((uint32_t)bz << 20);
}
__host__ __device__ inline void unpack_key(uint32_t k, int &bx, int &by, int &bz)
{
    bx = (int)(k & 1023u);
    by = (int)((k >> 10) & 1023u);
    bz = (int)((k >> 20) & 1023u);
}
__host__ __device__ inline uint32_t hash_key(uint32_t k)
{
    // murmur3 finaliser
    k ^= k >> 16;
    k *= 0x85ebca6bu;
    k ^= k >> 13;
    k *= 0xc2b2ae35u;
    k ^= k >> 16;
    return k;
}
__host__ __device__ inline uint64_t block_linear(const VolumeView &v, int bx, int by, int bz)
{
    // at most 1024 blocks per axis: the index fits in 30 bits
    return (uint64_t)(((uint32_t)bz * (uint32_t)v.nblk[1] + (uint32_t)by) * (uint32_t)v.nblk[0] + (uint32_t)bx);
}

// Lookup: slot or -1.
__device__ inline int32_t hash_find(const VolumeView &v, uint32_t key)
{
    uint32_t h = hash_key(key) & v.hash_mask;
    for (int p = 0; p < kMaxProbes; ++p) {
        unsigned long long e = v.hash[h];
        uint32_t k = (uint32_t)(e & 0xffffffffu);
        if (k == key) return (int32_t)(e >> 32);
        if (k == kEmptyKey) return -1;
        h = (h + 1) & v.hash_mask;
    }
    return -1;
}

// Insert a key that no other thread inserts concurrently and that is not in
// the table.  Returns the new pool slot, or -1 with a sticky flag set.
__device__ inline int32_t hash_insert_unique(const VolumeView &v, uint32_t key)
{
    uint32_t slot = atomicAdd(&v.state->pool_count, 1u);
    if (slot >= v.capacity) {
        atomicOr(&v.state->status, (uint32_t)TSDF_FLAG_POOL_FULL);
        return -1;
    }
    unsigned long long entry = ((unsigned long long)slot << 32) | key;
    v.pool_keys[slot] = key;
    uint32_t h = hash_key(key) & v.hash_mask;
    for (int p = 0; p < kMaxProbes; ++p) {
        unsigned long long prev = atomicCAS(&v.hash[h], kEmptyEntry, entry);
        if (prev == kEmptyEntry) return (int32_t)slot;
        if ((uint32_t)(prev & 0xffffffffu) == key) return (int32_t)(prev >> 32);
        h = (h + 1) & v.hash_mask;
    }
    // the slot stays reserved but holds no block: passes over the pool skip it
    v.pool_keys[slot] = kEmptyKey;
    atomicOr(&v.state->status, (uint32_t)TSDF_FLAG_HASH_FULL);
    return -1;
}

// Bounding box of a block's non-chi voxels, local coordinates 0..7: bits
// 0-8 the low corner (x, y, z, 3 bits each), bits 9-17 the high corner,
// bit 31 set when the box is not empty.  Boxes only grow (a voxel that
// returns to chi stays inside), so they stay conservative.
constexpr uint32_t kBoxValid = 1u << 31;

__host__ __device__ inline uint32_t box_make(int x0, int y0, int z0, int x1, int y1, int z1)
{
    return kBoxValid | (uint32_t)x0 | ((uint32_t)y0 << 3) | ((uint32_t)z0 << 6) | ((uint32_t)x1 << 9) |
           ((uint32_t)y1 << 12) | ((uint32_t)z1 << 15);
}

__host__ __device__ inline int box_lo(uint32_t b, int axis) { return (int)((b >> (3 * axis)) & 7u); }
__host__ __device__ inline int box_hi(uint32_t b, int axis) { return (int)((b >> (9 + 3 * axis)) & 7u); }

__host__ __device__ inline uint32_t box_union(uint32_t a, uint32_t b)
{
    if (!(a & kBoxValid)) return b;
    if (!(b & kBoxValid)) return a;
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        lo[k] = box_lo(a, k) < box_lo(b, k) ? box_lo(a, k) : box_lo(b, k);
        hi[k] = box_hi(a, k) > box_hi(b, k) ? box_hi(a, k) : box_hi(b, k);
    }
    return box_make(lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]);
}

// Box of the voxels of a wavefront's block that `zmask` (bit z: voxel
// (x, y, z) of this lane's column, lane = x + 8 y) marks; 0 when none.
__device__ inline uint32_t wave_box(uint32_t zmask)
{
    const unsigned long long L = __ballot(zmask != 0u);
    if (!L) return 0u;
    uint32_t zb = 0;
#pragma unroll
    for (int z = 0; z < 8; ++z) zb |= (__ballot((zmask >> z) & 1u) != 0ull ? 1u : 0u) << z;
    uint32_t xb = 0, yb = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const uint32_t row = (uint32_t)(L >> (8 * r)) & 0xffu;
        xb |= row;
        yb |= (row != 0u ? 1u : 0u) << r;
    }
    return box_make(__builtin_ctz(xb), __builtin_ctz(yb), __builtin_ctz(zb), 31 - __builtin_clz(xb),
                    31 - __builtin_clz(yb), 31 - __builtin_clz(zb & 0xffu));
}

// Largest pool: slot * 512 + voxel stays below 2^31 (32-bit pool offsets).
constexpr uint32_t kMaxCapacity = 1u << 22;
constexpr int32_t kIndexPositive = 1 << 30;   // dense index: every non-chi value of the block is > 0
constexpr int32_t kIndexSlotMask = kIndexPositive - 1;

// Order-preserving map float -> uint32 (for integer min over floats).
__host__ __device__ inline uint32_t order_key(float f)
{
    uint32_t b;
    memcpy(&b, &f, 4);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ inline float order_value(uint32_t k)
{
    uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    float f;
    memcpy(&f, &b, 4);
    return f;
}
constexpr uint32_t kKeyPosInf = 0xff800000u;   // order_key(+inf)
constexpr uint32_t kKeyZero = 0x80000000u;     // order_key(+0.0f)

// Wave-wide minimum.
__device__ inline uint32_t wave_min_u32(uint32_t x)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = min(x, (uint32_t)__shfl_xor((int)x, off));
    return x;
}

__device__ inline bool occupied(const VolumeView &v, int bx, int by, int bz)
{
    uint64_t b = block_linear(v, bx, by, bz);
    return (v.occupancy[b >> 5] >> (b & 31)) & 1u;
}

// ---- launchers (return hipError_t of the launch)
hipError_t launch_clear(const VolumeView &v, uint64_t words_total, uint32_t *base, hipStream_t s);
hipError_t launch_init_hash(const VolumeView &v, hipStream_t s);
hipError_t launch_frame_begin(const VolumeView &v, hipStream_t s);
hipError_t launch_prep(const VolumeView &v, const float *depth, const Camera &cam, const NoiseParams &noise,
                       hipStream_t s);
hipError_t launch_fuse(const VolumeView &v, const Camera &cam, hipStream_t s);
hipError_t launch_range(const VolumeView &v, const Camera &cam, uint32_t stamp, hipStream_t s);
hipError_t launch_count_bits(const uint32_t *bits, uint64_t words, unsigned long long *out, hipStream_t s);
hipError_t launch_march(const VolumeView &v, const Camera &cam, uint32_t stamp, int group, float4 *vertex,
                        float4 *normal, hipStream_t s, bool mark = false);
hipError_t launch_export(const VolumeView &v, int32_t *keys, void *T, void *P, uint32_t cap, hipStream_t s);
hipError_t launch_import(const VolumeView &v, const int32_t *keys, const void *T, const void *P, uint32_t n,
                         hipStream_t s);

// Host access to a volume for the batched path (volume.hip).  volume_view
// returns the device pointers and sizes; volume_enqueue prepares a volume
// for work that another path enqueues on `s` (remembers the stream, hands
// out the next raycast stamp when `stamp` is non-null) and returns
// TSDF_EFULL once a sticky device flag has been seen.
VolumeView volume_view(const tsdf_volume *vol);
tsdf_status volume_enqueue(tsdf_volume *vol, hipStream_t s, uint32_t *stamp);
// Records sticky device flags the caller has read back (later calls return TSDF_EFULL).
void volume_note_flags(tsdf_volume *vol, uint32_t flags);

}  // namespace tsdf

// Block eviction: the blocks outside a working box are copied out and
// removed, the volume shift that Section 8 names as future work.
//
//   count    evicted blocks among the allocated slots (the call returns
//            TSDF_ENOMEM before changing anything if they do not fit)
//   mark     one lane per slot: an evicted block is copied out; an
//            evicted slot below the new block count K is a hole, a kept slot
//            at or above K is a mover (there are as many of each)
//   move     one wavefront per mover: its voxels, key, bound and box go to a
//            hole, so the kept blocks end up in slots [0, K); a hole is only
//            written after the mark pass read it, and a mover is never a hole
//   rebuild  the pool counter becomes K; the hash table, the occupancy bits
//            and the dense index are cleared and refilled from the K blocks
#include <math.h>

#include "tsdf_internal.h"

namespace tsdf {
namespace {

struct EvictCounters {
    uint32_t evicted, exported, holes, movers;
    uint32_t pad[60];
};
static_assert(sizeof(EvictCounters) == 256, "counter line");

__device__ __forceinline__ bool inside_box(uint32_t key, int3 lo, int3 hi)
{
    int bx, by, bz;
    unpack_key(key, bx, by, bz);
    return bx >= lo.x && bx <= hi.x && by >= lo.y && by <= hi.y && bz >= lo.z && bz <= hi.z;
}

__global__ __launch_bounds__(256) void evict_count_kernel(VolumeView v, uint32_t n, int3 lo, int3 hi,
                                                          EvictCounters *c)
{
    for (uint32_t s = blockIdx.x * 256u + threadIdx.x; s < n; s += gridDim.x * 256u) {
        const bool out = !inside_box(v.pool_keys[s], lo, hi);
        const unsigned long long m = __ballot(out);
        if (out && __lane_id() == (uint32_t)(__ffsll((long long)m) - 1)) atomicAdd(&c->evicted, (uint32_t)__popcll(m));
    }
}

// One wavefront per 64 consecutive slots: each lane classifies one slot, the
// wavefront reserves its ranges of the output, hole and mover lists with one
// atomic each, then copies its evicted blocks one after the other (64 lanes
// per block, coalesced).
template <typename S>
__global__ __launch_bounds__(256) void evict_mark_kernel(VolumeView v, uint32_t n, uint32_t K, int3 lo, int3 hi,
                                                         int32_t *__restrict__ keys_out, S *__restrict__ T_out,
                                                         S *__restrict__ P_out, uint32_t *__restrict__ holes,
                                                         uint32_t *__restrict__ movers, EvictCounters *c)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    const uint32_t nw = gridDim.x * 4u;
    for (uint32_t base = (blockIdx.x * 4u + (threadIdx.x >> 6)) * 64u; base < n; base += nw * 64u) {
        const uint32_t s = base + lane;
        const bool valid = s < n;
        const uint32_t key = valid ? v.pool_keys[s] : 0u;
        const bool out = valid && !inside_box(key, lo, hi);
        const bool hole = out && s < K, mover = valid && !out && s >= K;
        const unsigned long long mo = __ballot(out), mh = __ballot(hole), mm = __ballot(mover);
        uint32_t e0 = 0, h0 = 0, m0 = 0;
        if (lane == 0) {
            if (mo) e0 = atomicAdd(&c->exported, (uint32_t)__popcll(mo));
            if (mh) h0 = atomicAdd(&c->holes, (uint32_t)__popcll(mh));
            if (mm) m0 = atomicAdd(&c->movers, (uint32_t)__popcll(mm));
        }
        e0 = __shfl(e0, 0);
        h0 = __shfl(h0, 0);
        m0 = __shfl(m0, 0);
        if (hole) holes[h0 + __popcll(mh & below)] = s;
        if (mover) movers[m0 + __popcll(mm & below)] = s;
        if (out) {
            const uint32_t e = e0 + (uint32_t)__popcll(mo & below);
            int b[3];
            unpack_key(key, b[0], b[1], b[2]);
            keys_out[3 * (size_t)e + 0] = b[0];
            keys_out[3 * (size_t)e + 1] = b[1];
            keys_out[3 * (size_t)e + 2] = b[2];
        }
        unsigned long long rest = mo;
        for (uint32_t r = 0; rest; ++r) {
            const int l = __ffsll((long long)rest) - 1;
            rest &= rest - 1ull;
            const uint32_t src = base + (uint32_t)l, dst = e0 + r;
            const S *srcT = (const S *)v.poolT + (size_t)src * kBlockVoxels;
            const S *srcP = (const S *)v.poolP + (size_t)src * kBlockVoxels;
            S *dT = T_out + (size_t)dst * kBlockVoxels;
            S *dP = P_out + (size_t)dst * kBlockVoxels;
#pragma unroll
            for (int q = 0; q < kBlockVoxels / 64; ++q) {
                dT[q * 64 + lane] = srcT[q * 64 + lane];
                dP[q * 64 + lane] = srcP[q * 64 + lane];
            }
        }
    }
}

template <typename S>
__global__ __launch_bounds__(256) void evict_move_kernel(VolumeView v, const uint32_t *__restrict__ holes,
                                                         const uint32_t *__restrict__ movers, const EvictCounters *c)
{
    const int lane = threadIdx.x & 63;
    const uint32_t nm = c->movers, nw = gridDim.x * 4u;
    for (uint32_t m = blockIdx.x * 4u + (threadIdx.x >> 6); m < nm; m += nw) {
        const uint32_t src = movers[m], dst = holes[m];
        S *T = (S *)v.poolT;
        S *P = (S *)v.poolP;
#pragma unroll
        for (int q = 0; q < kBlockVoxels / 64; ++q) {
            T[(size_t)dst * kBlockVoxels + q * 64 + lane] = T[(size_t)src * kBlockVoxels + q * 64 + lane];
            P[(size_t)dst * kBlockVoxels + q * 64 + lane] = P[(size_t)src * kBlockVoxels + q * 64 + lane];
        }
        if (lane == 0) {
            v.pool_keys[dst] = v.pool_keys[src];
            v.block_min[dst] = v.block_min[src];
            v.block_box[dst] = v.block_box[src];
        }
    }
}

__global__ void evict_fill_kernel(uint32_t *__restrict__ p, uint64_t n, uint32_t value)
{
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) p[i] = value;
}

__global__ void evict_set_count_kernel(DeviceState *st, uint32_t K) { st->pool_count = K; }

// Re-enters the K kept blocks: hash entry (slot << 32 | key), occupancy bit
// and dense-index entry (slot and sign flag, as the fusion writes them).
__global__ __launch_bounds__(256) void evict_rebuild_kernel(VolumeView v, uint32_t K)
{
    for (uint32_t s = blockIdx.x * 256u + threadIdx.x; s < K; s += gridDim.x * 256u) {
        const uint32_t key = v.pool_keys[s];
        const unsigned long long entry = ((unsigned long long)s << 32) | key;
        uint32_t h = hash_key(key) & v.hash_mask;
        bool placed = false;
        for (int p = 0; p < kMaxProbes && !placed; ++p) {
            placed = atomicCAS(&v.hash[h], kEmptyEntry, entry) == kEmptyEntry;
            h = (h + 1) & v.hash_mask;
        }
        if (!placed) atomicOr(&v.state->status, (uint32_t)TSDF_FLAG_HASH_FULL);
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        const uint64_t b = block_linear(v, bx, by, bz);
        atomicOr(&v.occupancy[b >> 5], 1u << (b & 31));
        if (v.block_index) v.block_index[b] = (int32_t)s | (v.block_min[s] > kKeyZero ? kIndexPositive : 0);
    }
}

constexpr uint32_t kEvictGrid = 2048;

uint64_t virtual_blocks(const VolumeView &v) { return (uint64_t)v.nblk[0] * v.nblk[1] * v.nblk[2]; }

}  // namespace
}  // namespace tsdf

using namespace tsdf;

extern "C" {

uint64_t tsdf_evict_workspace_bytes(const tsdf_volume *vol)
{
    if (!vol) return 0;
    const VolumeView v = volume_view(vol);
    return sizeof(EvictCounters) + 2 * (((uint64_t)v.capacity * 4 + 255) & ~(uint64_t)255);
}

tsdf_status tsdf_evict_blocks(tsdf_volume *vol, const int32_t lo[3], const int32_t hi[3], int32_t *keys_dev,
                              void *T_dev, void *P_dev, uint64_t cap, void *work_dev, uint64_t work_bytes,
                              uint64_t *n_out, hipStream_t stream)
{
    if (!vol || !lo || !hi || !n_out || !work_dev || work_bytes < tsdf_evict_workspace_bytes(vol) ||
        (cap > 0 && (!keys_dev || !T_dev || !P_dev)))
        return TSDF_EINVAL;
    tsdf_status st = volume_enqueue(vol, stream, nullptr);
    if (st != TSDF_OK) return st;
    const VolumeView v = volume_view(vol);
    const int3 blo = make_int3(lo[0], lo[1], lo[2]), bhi = make_int3(hi[0], hi[1], hi[2]);
    EvictCounters *c = (EvictCounters *)work_dev;
    const uint64_t list_bytes = ((uint64_t)v.capacity * 4 + 255) & ~(uint64_t)255;
    uint32_t *holes = (uint32_t *)((uint8_t *)work_dev + sizeof(EvictCounters));
    uint32_t *movers = (uint32_t *)((uint8_t *)work_dev + sizeof(EvictCounters) + list_bytes);

    DeviceState ds;
    hipError_t e = hipMemcpyAsync(&ds, v.state, sizeof(ds), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return TSDF_EHIP;
    *n_out = 0;
    if (ds.status != 0) {
        // a pool, hash or candidate overflow left the volume incomplete (and
        // possibly a reserved slot without a block): refuse, as later calls do
        volume_note_flags(vol, ds.status);
        return TSDF_EFULL;
    }
    const uint32_t n = ds.pool_count < v.capacity ? ds.pool_count : v.capacity;
    if (n == 0) return TSDF_OK;
    // count, and stop before any change if the evicted blocks do not fit
    hipLaunchKernelGGL(evict_fill_kernel, dim3(1), dim3(256), 0, stream, (uint32_t *)c, (uint64_t)64, 0u);
    hipLaunchKernelGGL(evict_count_kernel, dim3(kEvictGrid), dim3(256), 0, stream, v, n, blo, bhi, c);
    EvictCounters hc;
    e = hipGetLastError();   // a failed launch leaves the counters unwritten: stop before reading them
    if (e == hipSuccess) e = hipMemcpyAsync(&hc, c, sizeof(hc), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return TSDF_EHIP;
    const uint32_t E = hc.evicted;
    *n_out = E;
    if (E > cap) return TSDF_ENOMEM;
    if (E == 0) return TSDF_OK;
    const uint32_t K = n - E;
    // copy out, list holes and movers, move
    hipLaunchKernelGGL(evict_fill_kernel, dim3(1), dim3(256), 0, stream, (uint32_t *)c, (uint64_t)64, 0u);
    if (v.storage == TSDF_F16) {
        hipLaunchKernelGGL(evict_mark_kernel<__half>, dim3(kEvictGrid), dim3(256), 0, stream, v, n, K, blo, bhi,
                           keys_dev, (__half *)T_dev, (__half *)P_dev, holes, movers, c);
        hipLaunchKernelGGL(evict_move_kernel<__half>, dim3(kEvictGrid), dim3(256), 0, stream, v, holes, movers, c);
    } else {
        hipLaunchKernelGGL(evict_mark_kernel<float>, dim3(kEvictGrid), dim3(256), 0, stream, v, n, K, blo, bhi,
                           keys_dev, (float *)T_dev, (float *)P_dev, holes, movers, c);
        hipLaunchKernelGGL(evict_move_kernel<float>, dim3(kEvictGrid), dim3(256), 0, stream, v, holes, movers, c);
    }
    // rebuild the lookups from the K kept blocks
    hipLaunchKernelGGL(evict_set_count_kernel, dim3(1), dim3(1), 0, stream, v.state, K);
    const uint64_t hash_words = 2ull * ((uint64_t)v.hash_mask + 1);
    hipLaunchKernelGGL(evict_fill_kernel, dim3(kEvictGrid), dim3(256), 0, stream, (uint32_t *)v.hash, hash_words,
                       0xffffffffu);
    const uint64_t vb = virtual_blocks(v);
    hipLaunchKernelGGL(evict_fill_kernel, dim3(kEvictGrid), dim3(256), 0, stream, v.occupancy, (vb + 31) / 32, 0u);
    if (v.block_index)
        hipLaunchKernelGGL(evict_fill_kernel, dim3(kEvictGrid), dim3(256), 0, stream, (uint32_t *)v.block_index, vb,
                           0xffffffffu);
    hipLaunchKernelGGL(evict_rebuild_kernel, dim3(kEvictGrid), dim3(256), 0, stream, v, K);
    e = hipGetLastError();
    return e == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

}  // extern "C"

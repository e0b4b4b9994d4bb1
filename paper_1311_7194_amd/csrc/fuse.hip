// Fusion of one depth map into the block-sparse TSDF (Section 7).
//
//   frame_begin  reset the per-frame counters
//   prep         per pixel: validity, measurement variance, and the blocks
//                overlapping the pixel's frustum cell over [D - delta, D + delta]
//                (candidate blocks, deduplicated first in LDS per 16x16 tile,
//                then across the frame with a bit per virtual block)
//   fuse         one wavefront per candidate block: the 512 projective
//                measurements, a ballot for "any voxel not chi", lookup or
//                lock-free insertion of the block, then Algorithm 3 on every
//                voxel with a measurement
//
// The allocation rule is the Fig. 4 caption's: a block is allocated exactly
// when one of its voxels receives something other than chi.  Section 7.2
// lets blocks in view but off the surface update only when already
// allocated; with a voxel-exact measurement this is the same set of voxel
// updates, since such voxels get chi and are not touched.
#include "tsdf_internal.h"

namespace tsdf {

__global__ void frame_begin_kernel(DeviceState *st)
{
    st->cand_count = 0;
    st->new_blocks = 0;
    st->frame_updates = 0;
    st->frame_fresh_updates = 0;
    st->frames += 1;
}

hipError_t launch_frame_begin(const VolumeView &v, hipStream_t s)
{
    hipLaunchKernelGGL(frame_begin_kernel, dim3(1), dim3(1), 0, s, v.state);
    return hipGetLastError();
}

// ---------------------------------------------------------------- prep

constexpr int kTile = 16;             // 16x16 pixels per workgroup
constexpr int kLdsSet = 2048;         // LDS hash set of block keys
constexpr int kLdsList = 1024;        // unique keys held for the global pass

// Marks `key` as a candidate of this frame; the first marker appends it to
// the candidate list.  Called by active lanes of one wavefront.
__device__ inline void global_candidate(const VolumeView &v, uint32_t key)
{
    int bx, by, bz;
    unpack_key(key, bx, by, bz);
    uint64_t b = block_linear(v, bx, by, bz);
    uint32_t bit = 1u << (b & 31);
    uint32_t old = atomicOr(&v.cand_bits[b >> 5], bit);
    bool fresh = !(old & bit);
    unsigned long long m = __ballot(fresh);
    if (!m) return;
    int lane = __lane_id();
    int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(&v.state->cand_count, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if (fresh) {
        uint32_t idx = base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (idx < v.max_candidates) {
            v.cand_list[idx] = key;
        } else {
            atomicOr(&v.state->status, (uint32_t)TSDF_FLAG_CAND_FULL);
            atomicAnd(&v.cand_bits[b >> 5], ~bit);
        }
    }
}

__device__ inline float measurement_variance(const NoiseParams &noise, float D, float inv_delta)
{
    if (noise.kind == TSDF_NOISE_CONSTANT) return noise.coeff;
    float r = noise.coeff * D * D * inv_delta;   // sigma / delta
    return r * r;
}

__global__ __launch_bounds__(256) void prep_kernel(VolumeView v, const float *__restrict__ depth, Camera cam,
                                                   NoiseParams noise)
{
    __shared__ uint32_t set[kLdsSet];
    __shared__ uint32_t list[kLdsList];
    __shared__ uint32_t n_list;
    const int tid = threadIdx.x;
    for (int k = tid; k < kLdsSet; k += 256) set[k] = kEmptyKey;
    if (tid == 0) n_list = 0;
    __syncthreads();

    const int i = blockIdx.x * kTile + (tid & (kTile - 1));
    const int j = blockIdx.y * kTile + (tid / kTile);
    const bool in_image = i < cam.width && j < cam.height;
    float D = in_image ? depth[(size_t)j * cam.width + i] : 0.0f;
    const bool valid = in_image && D > 0.0f && isfinite(D);
    const float inv_delta_f = (float)v.inv_delta;
    if (in_image) {
        float ph = valid ? measurement_variance(noise, D, inv_delta_f) : 0.0f;
        v.pixmap[(size_t)j * cam.width + i] = make_float2(valid ? D : 0.0f, ph);
    }

    if (valid) {
        // world box of the frustum cell (pixel square x depth range)
        const double z0 = fmax((double)D - v.delta, 0.0), z1 = (double)D + v.delta;
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double u = i + ((k & 1) ? 0.5 : -0.5);
            const double w = j + ((k & 2) ? 0.5 : -0.5);
            const double z = (k & 4) ? z1 : z0;
            const double xc = (u - cam.cx) / cam.fx * z, yc = (w - cam.cy) / cam.fy * z;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double xw = cam.R[3 * a] * xc + cam.R[3 * a + 1] * yc + cam.R[3 * a + 2] * z + cam.t[a];
                lo[a] = fmin(lo[a], xw);
                hi[a] = fmax(hi[a], xw);
            }
        }
        const double pad = 0.01 * v.vs;
        int b0[3], b1[3];
        bool empty = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double g0 = ceil((lo[a] - pad - v.origin[a]) * v.inv_vs - 0.5);
            double g1 = floor((hi[a] + pad - v.origin[a]) * v.inv_vs - 0.5);
            g0 = fmax(g0, 0.0);
            g1 = fmin(g1, (double)(v.dims[a] - 1));
            empty |= g0 > g1;
            b0[a] = (int)g0 >> 3;
            b1[a] = (int)g1 >> 3;
        }
        if (!empty) {
            for (int bz = b0[2]; bz <= b1[2]; ++bz)
                for (int by = b0[1]; by <= b1[1]; ++by)
                    for (int bx = b0[0]; bx <= b1[0]; ++bx) {
                        const uint32_t key = pack_key(bx, by, bz);
                        uint32_t h = hash_key(key) & (kLdsSet - 1);
                        bool placed = false;
                        for (int p = 0; p < 64; ++p) {
                            uint32_t prev = atomicCAS(&set[h], kEmptyKey, key);
                            if (prev == kEmptyKey) {
                                uint32_t slot = atomicAdd(&n_list, 1u);
                                if (slot < (uint32_t)kLdsList) {
                                    list[slot] = key;
                                    placed = true;
                                }
                                break;
                            }
                            if (prev == key) {
                                placed = true;
                                break;
                            }
                            h = (h + 1) & (kLdsSet - 1);
                        }
                        // LDS set or list exhausted: go straight to the frame-wide dedup
                        if (!placed) {
                            // single-lane path: emulate with a one-lane wave call
                            uint64_t b = block_linear(v, bx, by, bz);
                            uint32_t bit = 1u << (b & 31);
                            uint32_t old = atomicOr(&v.cand_bits[b >> 5], bit);
                            if (!(old & bit)) {
                                uint32_t idx = atomicAdd(&v.state->cand_count, 1u);
                                if (idx < v.max_candidates) {
                                    v.cand_list[idx] = key;
                                } else {
                                    atomicOr(&v.state->status, (uint32_t)TSDF_FLAG_CAND_FULL);
                                    atomicAnd(&v.cand_bits[b >> 5], ~bit);
                                }
                            }
                        }
                    }
        }
    }
    __syncthreads();
    const uint32_t n = min(n_list, (uint32_t)kLdsList);
    for (uint32_t k = tid; k < n; k += 256) global_candidate(v, list[k]);
}

hipError_t launch_prep(const VolumeView &v, const float *depth, const Camera &cam, const NoiseParams &noise,
                       hipStream_t s)
{
    dim3 grid((cam.width + kTile - 1) / kTile, (cam.height + kTile - 1) / kTile);
    hipLaunchKernelGGL(prep_kernel, grid, dim3(256), 0, s, v, depth, cam, noise);
    return hipGetLastError();
}

// ---------------------------------------------------------------- fuse

// Projective measurement of one voxel given the lane-constant partial sums
// of x_c = R^T (x - t).  The operation order repeats the definition exactly
// (no contraction), so the decisions (nearest pixel, |s| <= delta) are the
// defined double-precision ones bit for bit.
struct LaneGeom {
    double ax, ay, az;   // R[0][k]*dx + R[1][k]*dy for k = x, y, z
};

__device__ __forceinline__ bool measure_voxel(const VolumeView &v, const Camera &cam, const LaneGeom &g, int gz,
                                              const float2 *__restrict__ pixmap, float &Tk, float &pk)
{
#pragma clang fp contract(off)
    const double pz = v.origin[2] + ((double)gz + 0.5) * v.vs;
    const double dz = pz - cam.t[2];
    const double xc = g.ax + cam.R[6] * dz;
    const double yc = g.ay + cam.R[7] * dz;
    const double zc = g.az + cam.R[8] * dz;
    if (!(zc > 0.0)) return false;
    const double u = cam.fx * xc / zc + cam.cx;
    const double w = cam.fy * yc / zc + cam.cy;
    const double fu = floor(u + 0.5);
    const double fw = floor(w + 0.5);
    if (!(fu >= 0.0 && fu < (double)cam.width && fw >= 0.0 && fw < (double)cam.height)) return false;
    const float2 pm = pixmap[(size_t)(int)fw * cam.width + (int)fu];
    if (!(pm.x > 0.0f)) return false;
    const double s = (double)pm.x - zc;
    if (!(fabs(s) <= v.delta)) return false;
    Tk = (float)(s * v.inv_delta);
    pk = pm.y;
    return true;
}

__device__ __forceinline__ void kalman(float &T, float &P, float Tk, float pk, float q)
{
    // Algorithm 3 in normalised units; chi is any |T| > 1
    if (fabsf(T) > 1.0f) {
        T = Tk;
        P = pk;
    } else {
        P = P + q;
        const float K = P / (P + pk);
        T = T + K * (Tk - T);
        P = (1.0f - K) * P;
    }
    if (fabsf(T) > 1.0f) T = kChi;
}

template <typename S>
__device__ __forceinline__ float load_s(const S *p);
template <>
__device__ __forceinline__ float load_s<float>(const float *p) { return *p; }
template <>
__device__ __forceinline__ float load_s<__half>(const __half *p) { return __half2float(*p); }
template <typename S>
__device__ __forceinline__ void store_s(S *p, float x);
template <>
__device__ __forceinline__ void store_s<float>(float *p, float x) { *p = x; }
template <>
__device__ __forceinline__ void store_s<__half>(__half *p, float x) { *p = __float2half_rn(x); }

template <typename S>
__global__ __launch_bounds__(256) void fuse_kernel(VolumeView v, Camera cam)
{
    const int lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * 4u;
    const uint32_t ncand = min(v.state->cand_count, v.max_candidates);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&v.state->total_candidates, (unsigned long long)ncand);
    const int lx = lane & 7, ly = lane >> 3;
    const float2 *__restrict__ pixmap = v.pixmap;
    S *__restrict__ poolT = (S *)v.poolT;
    S *__restrict__ poolP = (S *)v.poolP;

    for (uint32_t c = wave; c < ncand; c += nwaves) {
        const uint32_t key = v.cand_list[c];
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        LaneGeom g;
        {
#pragma clang fp contract(off)
            const double px = v.origin[0] + ((double)(bx * 8 + lx) + 0.5) * v.vs;
            const double py = v.origin[1] + ((double)(by * 8 + ly) + 0.5) * v.vs;
            const double dx = px - cam.t[0];
            const double dy = py - cam.t[1];
            g.ax = cam.R[0] * dx + cam.R[3] * dy;
            g.ay = cam.R[1] * dx + cam.R[4] * dy;
            g.az = cam.R[2] * dx + cam.R[5] * dy;
        }
        float Tk[8], pk[8];
        uint32_t vmask = 0;
#pragma unroll
        for (int z = 0; z < 8; ++z) {
            Tk[z] = kChi;
            pk[z] = 0.0f;
            if (measure_voxel(v, cam, g, bz * 8 + z, pixmap, Tk[z], pk[z])) vmask |= 1u << z;
        }
        if (lane == 0) {
            uint64_t b = block_linear(v, bx, by, bz);
            atomicAnd(&v.cand_bits[b >> 5], ~(1u << (b & 31)));
        }
        const unsigned long long any = __ballot(vmask != 0);
        if (!any) continue;

        int32_t slot = -1;
        int fresh = 0;
        if (lane == 0) {
            slot = hash_find(v, key);
            if (slot < 0) {
                slot = hash_insert_unique(v, key);
                if (slot >= 0) {
                    fresh = 1;
                    uint64_t b = block_linear(v, bx, by, bz);
                    atomicOr(&v.occupancy[b >> 5], 1u << (b & 31));
                    atomicAdd(&v.state->new_blocks, 1u);
                    atomicAdd(&v.state->total_new_blocks, 1ull);
                }
            }
        }
        slot = __shfl(slot, 0);
        fresh = __shfl(fresh, 0);
        if (slot < 0) continue;

        S *bt = poolT + (size_t)slot * kBlockVoxels + lane;
        S *bp = poolP + (size_t)slot * kBlockVoxels + lane;
        if (fresh) {
#pragma unroll
            for (int z = 0; z < 8; ++z) {
                const bool m = (vmask >> z) & 1u;
                store_s(bt + 64 * z, m ? Tk[z] : kChi);
                store_s(bp + 64 * z, m ? pk[z] : 0.0f);
            }
        } else {
#pragma unroll
            for (int z = 0; z < 8; ++z) {
                if ((vmask >> z) & 1u) {
                    float T = load_s(bt + 64 * z);
                    float P = load_s(bp + 64 * z);
                    kalman(T, P, Tk[z], pk[z], v.q_hat);
                    store_s(bt + 64 * z, T);
                    store_s(bp + 64 * z, P);
                }
            }
        }
        // count Algorithm 3 executions: wave sum of popcounts
        uint32_t cnt = __popc(vmask);
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
        if (lane == 0) {
            atomicAdd(&v.state->frame_updates, (unsigned long long)cnt);
            atomicAdd(&v.state->total_updates, (unsigned long long)cnt);
            if (fresh) {
                atomicAdd(&v.state->frame_fresh_updates, (unsigned long long)cnt);
                atomicAdd(&v.state->total_fresh_updates, (unsigned long long)cnt);
            }
        }
    }
}

hipError_t launch_fuse(const VolumeView &v, const Camera &cam, hipStream_t s)
{
    // persistent grid: enough waves to fill 256 CUs several times over
    uint32_t want = (v.max_candidates + 3) / 4;
    uint32_t blocks = want < 4096u ? want : 4096u;
    if (blocks == 0) blocks = 1;
    if (v.storage == TSDF_F16)
        hipLaunchKernelGGL(fuse_kernel<__half>, dim3(blocks), dim3(256), 0, s, v, cam);
    else
        hipLaunchKernelGGL(fuse_kernel<float>, dim3(blocks), dim3(256), 0, s, v, cam);
    return hipGetLastError();
}

}  // namespace tsdf

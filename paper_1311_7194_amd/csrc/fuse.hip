// Fusion of one depth map into the block-sparse TSDF (Section 7).
//
//   frame_begin  reset the per-frame counters
//   prep         per pixel: validity, measurement variance, and the blocks
//                that the pixel's frustum cell over [D - delta, D + delta] may
//                reach (candidate blocks, deduplicated first in LDS per 16x16
//                tile, then across the frame with a bit per virtual block)
//   fuse         one wavefront per candidate block: the 512 projective
//                measurements, a ballot for "any voxel not chi", lookup or
//                lock-free insertion of the block, then Algorithm 3 on every
//                voxel with a measurement
//
// The allocation rule is the Fig. 4 caption's: a block is allocated exactly
// when one of its voxels receives something other than chi.  Section 7.2
// lets blocks in view but off the surface update only when already
// allocated; with a voxel-exact measurement this is the same set of voxel
// updates, since such voxels get chi and are not touched.  The paper reads
// the sampled block list back to the CPU for allocation; here allocation
// stays on the device (atomic pool counter, lock-free hash).
#include "fuse_device.h"

namespace tsdf {

__global__ void frame_begin_kernel(DeviceState *st, Counters *ctr) { frame_begin_body(st, ctr, threadIdx.x); }

hipError_t launch_frame_begin(const VolumeView &v, hipStream_t s)
{
    hipLaunchKernelGGL(frame_begin_kernel, dim3(1), dim3(kCtrLanes), 0, s, v.state, v.ctr);
    return hipGetLastError();
}

template <bool kMlp>
__global__ __launch_bounds__(256) void prep_kernel(VolumeView v, const float *__restrict__ depth, Camera cam,
                                                   NoiseParams noise)
{
    prep_body<kMlp>(v, depth, cam, noise, blockIdx.x, blockIdx.y);
}

hipError_t launch_prep(const VolumeView &v, const float *depth, const Camera &cam, const NoiseParams &noise,
                       hipStream_t s)
{
    dim3 grid((cam.width + kTile - 1) / kTile, (cam.height + kTile - 1) / kTile);
    if (noise.kind == TSDF_NOISE_MLP)
        hipLaunchKernelGGL(prep_kernel<true>, grid, dim3(256), 0, s, v, depth, cam, noise);
    else
        hipLaunchKernelGGL(prep_kernel<false>, grid, dim3(256), 0, s, v, depth, cam, noise);
    return hipGetLastError();
}

template <typename S>
// five waves per SIMD: a few spilled registers cost less than the lost latency hiding
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void fuse_kernel(VolumeView v, Camera cam, FuseCam fc)
{
    const int lane = threadIdx.x & 63;
    const uint32_t wave = blockIdx.x * 4u + (threadIdx.x >> 6);
    const uint32_t nwaves = gridDim.x * 4u;
    const uint32_t ncand = min(v.state->cand_count, v.max_candidates);
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&v.state->total_candidates, (unsigned long long)ncand);
    FuseAcc acc;
    // the next candidate's key is loaded one block ahead
    uint32_t key = wave < ncand ? v.cand_list[wave] : 0u;
    for (uint32_t c = wave; c < ncand; c += nwaves) {
        const uint32_t next = c + nwaves < ncand ? v.cand_list[c + nwaves] : 0u;
        fuse_block<S>(v, cam, fc, key, lane, acc);
        key = next;
    }
    fuse_flush(v, acc, wave, lane);
}

hipError_t launch_fuse(const VolumeView &v, const Camera &cam, hipStream_t s)
{
    // persistent grid of 2560 workgroups: two rounds of resident waves at
    // five per SIMD on 256 CUs (one round or 3.2 rounds measured slower)
    uint32_t want = (v.max_candidates + 3) / 4;
    uint32_t blocks = want < kFuseGrid ? want : kFuseGrid;
    if (blocks == 0) blocks = 1;
    const FuseCam fc = make_fuse_cam(v, cam);
    if (v.storage == TSDF_F16)
        hipLaunchKernelGGL(fuse_kernel<__half>, dim3(blocks), dim3(256), 0, s, v, cam, fc);
    else
        hipLaunchKernelGGL(fuse_kernel<float>, dim3(blocks), dim3(256), 0, s, v, cam, fc);
    return hipGetLastError();
}

}  // namespace tsdf

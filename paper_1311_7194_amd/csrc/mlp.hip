// Learned measurement-noise model: features, inference and training kernels.
//
// Training minimises the Gaussian negative log-likelihood 1/2 (s + r^2 e^-s)
// of residuals r = D - Z between a frame's measured depth D and the depth Z
// of the fused surface raycast from that frame's pose, with s = log sigma^2
// predicted from the pixel's features.  Forward, backward and the Adam update
// are hand-written: the two layer-2 products of the backward pass run on the
// matrix cores like the forward product.
#include "tsdf_internal.h"
#include "mlp_device.h"
#include "mlp_features.h"
#include "tsdf_mlp.h"

namespace tsdf {

// ---------------------------------------------------------------- features

__global__ __launch_bounds__(256) void features_kernel(const float *__restrict__ depth, int W, int H, double fx,
                                                       double fy, double cx, double cy, float4 *__restrict__ feat,
                                                       uint8_t *__restrict__ valid)
{
    __shared__ FeatLds L;
    const int i0 = blockIdx.x * kFeatTile, j0 = blockIdx.y * kFeatTile;
    float f[4];
    const bool ok = tile_features(L, depth, W, H, fx, fy, cx, cy, i0, j0, threadIdx.x, f);
    const int i = i0 + threadIdx.x % kFeatTile, j = j0 + threadIdx.x / kFeatTile;
    if (i < W && j < H) {
        feat[(size_t)j * W + i] = make_float4(f[0], f[1], f[2], f[3]);
        valid[(size_t)j * W + i] = ok ? 1 : 0;
    }
}

// ---------------------------------------------------------------- forward

__global__ __launch_bounds__(256) void forward_kernel(const uint16_t *__restrict__ params,
                                                      const float4 *__restrict__ x, int64_t n, float *__restrict__ s)
{
    __shared__ MlpParamsLds P;
    __shared__ MlpInferLds Wl[4];
    mlp_stage_params(P, params, threadIdx.x, 256);
    __syncthreads();
    const int64_t k = blockIdx.x * 256ll + threadIdx.x;
    float4 xv = k < n ? x[k] : make_float4(0.f, 0.f, 0.f, 0.f);
    const float xa[4] = {xv.x, xv.y, xv.z, xv.w};
    // the same forward pass as the integration path
    const float out = mlp_infer_wave(P, params, Wl[threadIdx.x >> 6], xa, threadIdx.x & 63);
    if (k < n) s[k] = out;
}

// ---------------------------------------------------------------- training

// Wave sum of a float (butterfly; every lane ends with the total).
__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Sample index of position k in the epoch's visiting order: an affine
// permutation k -> (a k + b) mod n with a coprime to n (chosen by the host).
// (a < n and k < n <= 2^31 keep a k + b inside 64 bits).
__device__ __forceinline__ int64_t visit(int64_t k, int64_t n, uint64_t a, uint64_t b)
{
    return (int64_t)(((uint64_t)a * (uint64_t)(k % n) + b) % (uint64_t)n);
}

constexpr int kTrainWaves = 2;   // 128 samples per workgroup keeps LDS under 64 KiB

struct TrainLds {
    MlpParamsLds P;
    MlpWaveLds wave[kTrainWaves];              // forward scratch; t3 then holds dL/dh1, h1 then dW2
    uint16_t e2[kTrainWaves][64][kMlpHidden + 4];   // bf16(dL/da2) per sample
    float ds[kTrainWaves][64];
    float red[kTrainWaves][kMlpHidden * kMlpIn + 3 * kMlpHidden + 2];
};

// One workgroup = 128 samples of the batch; writes the workgroup's summed
// gradient (1249 values) and loss into partial[blockIdx.x].
__global__ __launch_bounds__(128) void train_kernel(const uint16_t *__restrict__ params,
                                                    const float4 *__restrict__ x, const float *__restrict__ r,
                                                    int64_t n_samples, int64_t first, int64_t batch, uint64_t pa,
                                                    uint64_t pb, float *__restrict__ partial)
{
    __shared__ TrainLds S;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NT = 64 * kTrainWaves;
    mlp_stage_params(S.P, params, tid, NT);
    __syncthreads();
    const int64_t kb = blockIdx.x * (int64_t)NT + tid;   // position inside the batch
    const bool live = kb < batch;
    float xa[4] = {0.f, 0.f, 0.f, 0.f}, rr = 0.f;
    if (live) {
        const int64_t idx = visit(first + kb, n_samples, pa, pb);
        const float4 xv = x[idx];
        xa[0] = xv.x;
        xa[1] = xv.y;
        xa[2] = xv.z;
        xa[3] = xv.w;
        rr = r[idx];
    }
    float a2[2][16];
    const float s = mlp_forward_wave(S.P, params + MLP_W2, S.wave[wv], xa, lane, a2);
    const float e = __expf(-s);
    const float loss = live ? 0.5f * (s + rr * rr * e) : 0.0f;
    const float ds = live ? 0.5f * (1.0f - rr * rr * e) : 0.0f;
    S.ds[wv][lane] = ds;
    __syncthreads();

    // output layer and dL/da2 in the accumulator layout (lane: unit o = lane % 32)
    const int col = lane & 31;
    const float w3 = S.P.p[MLP_W3 + col];
    float gW3 = 0.f, gb2 = 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int row = 32 * t + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
            const float dsr = S.ds[wv][row];
            const float h2 = bf16_round(silu(a2[t][q]));
            const float da2 = dsr * w3 * silu_grad(a2[t][q]);
            gW3 += dsr * h2;
            gb2 += da2;
            S.e2[wv][row][col] = bf16_bits(da2);
        }
    __syncthreads();

    // dW2[o][i] = sum_m e2[m][o] h1[m][i]: M = o, N = i, K = samples (16 per step)
    f32x16_t w2c;
    {
        const int kh = 8 * (lane >> 5);
        f32x16_t c = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            i16x8_t a, b;
#pragma unroll
            for (int el = 0; el < 8; ++el) {
                a[el] = (short)S.e2[wv][16 * kk + kh + el][col];
                b[el] = (short)S.wave[wv].h1[16 * kk + kh + el][col];
            }
            c = mfma_bf16_k16(a, b, c);
        }
        w2c = c;
    }
    // dh1[m][i] = sum_o e2[m][o] W2[o][i]: M = samples (two tiles), N = i, K = o
    {
        const int kh = 8 * (lane >> 5);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            f32x16_t c = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                i16x8_t a, b;
#pragma unroll
                for (int el = 0; el < 8; ++el) {
                    a[el] = (short)S.e2[wv][32 * t + col][16 * kk + kh + el];
                    b[el] = (short)params[MLP_W2 + (16 * kk + kh + el) * kMlpHidden + col];
                }
                c = mfma_bf16_k16(a, b, c);
            }
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int m = 32 * t + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
                S.wave[wv].t3[m][col] = c[q];   // dL/dh1, transposed to one sample per row
            }
        }
    }
    __syncthreads();   // every wavefront has read h1: its space now takes the dW2 tile
    float *w2part = reinterpret_cast<float *>(&S.wave[wv].h1[0][0]);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int o = 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        w2part[o * kMlpHidden + col] = w2c[q];
    }

    // layer 1, one sample per lane: da1 = dh1 silu'(a1); dW1 = da1 x0^T, db1 = da1
    float x0[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) x0[i] = bf16_round(xa[i]);
    float g1[kMlpHidden * kMlpIn], gb1[kMlpHidden];
#pragma unroll
    for (int o = 0; o < kMlpHidden; ++o) {
        float a = S.P.p[MLP_B1 + o];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) a += S.P.p[MLP_W1 + o * kMlpIn + i] * x0[i];
        const float da1 = S.wave[wv].t3[lane][o] * silu_grad(a);
        gb1[o] = da1;
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) g1[o * kMlpIn + i] = da1 * x0[i];
    }
    // wave reductions, then across the 4 wavefronts
    float *red = S.red[wv];
#pragma unroll
    for (int k = 0; k < kMlpHidden * kMlpIn; ++k) {
        const float v = wave_sum(g1[k]);
        if (lane == 0) red[k] = v;
    }
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k) {
        const float v = wave_sum(gb1[k]);
        if (lane == 0) red[kMlpHidden * kMlpIn + k] = v;
    }
    {
        // gW3 and gb2 live in lanes o and o + 32 (two row halves)
        const float w3s = gW3 + __shfl_xor(gW3, 32), b2s = gb2 + __shfl_xor(gb2, 32);
        if (lane < 32) {
            red[kMlpHidden * kMlpIn + kMlpHidden + lane] = b2s;
            red[kMlpHidden * kMlpIn + 2 * kMlpHidden + lane] = w3s;
        }
        const float b3s = wave_sum(ds), ls = wave_sum(loss);
        if (lane == 0) {
            red[kMlpHidden * kMlpIn + 3 * kMlpHidden] = b3s;
            red[kMlpHidden * kMlpIn + 3 * kMlpHidden + 1] = ls;
        }
    }
    __syncthreads();
    float *out = partial + (size_t)blockIdx.x * kMlpParamsPadded;
    for (int k = tid; k < kMlpHidden * kMlpIn + 3 * kMlpHidden + 2; k += NT) {
        float v = 0.0f;
#pragma unroll
        for (int w = 0; w < kTrainWaves; ++w) v += S.red[w][k];
        int dst;
        if (k < 128) dst = MLP_W1 + k;
        else if (k < 160) dst = MLP_B1 + (k - 128);
        else if (k < 192) dst = MLP_B2 + (k - 160);
        else if (k < 224) dst = MLP_W3 + (k - 192);
        else if (k == 224) dst = MLP_B3;
        else dst = kMlpParams;   // loss, stored in the padding
        out[dst] = v;
    }
    for (int k = tid; k < kMlpHidden * kMlpHidden; k += NT) {
        float v = 0.0f;
#pragma unroll
        for (int w = 0; w < kTrainWaves; ++w) v += reinterpret_cast<const float *>(&S.wave[w].h1[0][0])[k];
        out[MLP_W2 + k] = v;
    }
}

// grad[p] = (sum over workgroups of partial[wg][p]) / batch; loss likewise.
__global__ void reduce_kernel(const float *__restrict__ partial, int n_wg, int64_t batch, float *__restrict__ grad,
                              float *__restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kMlpParams) return;
    double acc = 0.0;
    for (int w = 0; w < n_wg; ++w) acc += partial[(size_t)w * kMlpParamsPadded + p];
    if (p < kMlpParams) grad[p] = (float)(acc / (double)batch);
    else if (loss) loss[0] = (float)(acc / (double)batch);
}

// Adam on float32 master weights; the bf16 parameters are their rounding.
__global__ void adam_kernel(float *__restrict__ master, float *__restrict__ m, float *__restrict__ v,
                            const float *__restrict__ grad, uint16_t *__restrict__ params, int step, float lr,
                            float beta1, float beta2, float eps)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = grad[p];
    const float mn = beta1 * m[p] + (1.0f - beta1) * g;
    const float vn = beta2 * v[p] + (1.0f - beta2) * g * g;
    m[p] = mn;
    v[p] = vn;
    const float mh = mn / (1.0f - powf(beta1, (float)step));
    const float vh = vn / (1.0f - powf(beta2, (float)step));
    const float w = master[p] - lr * mh / (sqrtf(vh) + eps);
    master[p] = w;
    params[p] = bf16_bits(w);
}

// Training samples of one frame: pixels with a measurement, valid features
// and a raycast hit; residual r = D - (camera z of the hit).  Pass 1 counts
// per workgroup, pass 2 scans the counts, pass 3 writes in pixel order.
__device__ __forceinline__ bool sample_of(const float *depth, const float4 *feat, const uint8_t *valid,
                                          const float4 *vertex, const Camera &cam, size_t k, float &res)
{
    const float D = depth[k];
    if (!(D > 0.0f) || !isfinite(D) || !valid[k]) return false;
    const float4 vt = vertex[k];
    if (!(vt.w > 0.0f)) return false;
    const double z = cam.R[2] * ((double)vt.x - cam.t[0]) + cam.R[5] * ((double)vt.y - cam.t[1]) +
                     cam.R[8] * ((double)vt.z - cam.t[2]);
    res = (float)((double)D - z);
    return true;
}

__global__ __launch_bounds__(256) void sample_count_kernel(const float *depth, const float4 *feat,
                                                           const uint8_t *valid, const float4 *vertex, Camera cam,
                                                           int64_t n, uint32_t *counts)
{
    const size_t k = blockIdx.x * 256ull + threadIdx.x;
    float res;
    const bool ok = k < (size_t)n && sample_of(depth, feat, valid, vertex, cam, k, res);
    const int c = __syncthreads_count(ok);
    if (threadIdx.x == 0) counts[blockIdx.x] = (uint32_t)c;
}

__global__ void scan_kernel(uint32_t *counts, int nblocks, uint64_t *base, uint64_t *total)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t acc = total[0];
    for (int b = 0; b < nblocks; ++b) {
        base[b] = acc;
        acc += counts[b];
    }
    total[0] = acc;
}

__global__ __launch_bounds__(256) void sample_write_kernel(const float *depth, const float4 *feat,
                                                           const uint8_t *valid, const float4 *vertex, Camera cam,
                                                           int64_t n, const uint64_t *base, int64_t cap,
                                                           float4 *xout, float *rout)
{
    __shared__ uint32_t wave_counts[4];
    const size_t k = blockIdx.x * 256ull + threadIdx.x;
    float res = 0.0f;
    const bool ok = k < (size_t)n && sample_of(depth, feat, valid, vertex, cam, k, res);
    const unsigned long long m = __ballot(ok);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) wave_counts[wv] = (uint32_t)__popcll(m);
    __syncthreads();
    uint64_t off = base[blockIdx.x];
    for (int w = 0; w < wv; ++w) off += wave_counts[w];
    off += (uint64_t)__popcll(m & ((1ull << lane) - 1ull));
    if (ok && (int64_t)off < cap) {
        xout[off] = feat[k];
        rout[off] = res;
    }
}

}  // namespace tsdf

using namespace tsdf;

extern "C" {

tsdf_status tsdf_mlp_features(const float *depth_dev, const tsdf_intrinsics *K, float *feat_dev, uint8_t *valid_dev,
                              hipStream_t stream)
{
    if (!depth_dev || !K || !feat_dev || !valid_dev || !(K->fx > 0) || !(K->fy > 0) || K->width <= 0 ||
        K->height <= 0)
        return TSDF_EINVAL;
    dim3 grid((K->width + kFeatTile - 1) / kFeatTile, (K->height + kFeatTile - 1) / kFeatTile);
    hipLaunchKernelGGL(features_kernel, grid, dim3(256), 0, stream, depth_dev, K->width, K->height, K->fx, K->fy,
                       K->cx, K->cy, (float4 *)feat_dev, valid_dev);
    return hipGetLastError() == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

tsdf_status tsdf_mlp_forward(const void *params_dev, const float *x_dev, int64_t n, float *s_dev, hipStream_t stream)
{
    if (!params_dev || n < 0 || (n > 0 && (!x_dev || !s_dev))) return TSDF_EINVAL;
    if (n == 0) return TSDF_OK;
    dim3 grid((unsigned)((n + 255) / 256));
    hipLaunchKernelGGL(forward_kernel, grid, dim3(256), 0, stream, (const uint16_t *)params_dev,
                       (const float4 *)x_dev, n, s_dev);
    return hipGetLastError() == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

uint64_t tsdf_mlp_workspace_bytes(int64_t batch)
{
    if (batch <= 0) return 0;
    return (uint64_t)((batch + 64 * kTrainWaves - 1) / (64 * kTrainWaves)) * kMlpParamsPadded * sizeof(float);
}

tsdf_status tsdf_mlp_loss_grad(const void *params_dev, const float *x_dev, const float *r_dev, int64_t n_samples,
                               int64_t first, int64_t batch, uint64_t perm_a, uint64_t perm_b, void *workspace_dev,
                               float *grad_dev, float *loss_dev, hipStream_t stream)
{
    if (!params_dev || !x_dev || !r_dev || !workspace_dev || !grad_dev || n_samples <= 0 || batch <= 0 || first < 0)
        return TSDF_EINVAL;
    if (perm_a == 0 || perm_a >= (uint64_t)n_samples || perm_b >= (uint64_t)n_samples || n_samples > (1ll << 31))
        return TSDF_EINVAL;
    const int n_wg = (int)((batch + 64 * kTrainWaves - 1) / (64 * kTrainWaves));
    hipLaunchKernelGGL(train_kernel, dim3(n_wg), dim3(64 * kTrainWaves), 0, stream, (const uint16_t *)params_dev,
                       (const float4 *)x_dev, r_dev, n_samples, first, batch, perm_a, perm_b, (float *)workspace_dev);
    if (hipGetLastError() != hipSuccess) return TSDF_EHIP;
    hipLaunchKernelGGL(reduce_kernel, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, stream,
                       (const float *)workspace_dev, n_wg, batch, grad_dev, loss_dev);
    return hipGetLastError() == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

tsdf_status tsdf_mlp_adam_step(float *master_dev, float *m_dev, float *v_dev, const float *grad_dev, void *params_dev,
                               int32_t step, float lr, float beta1, float beta2, float eps, hipStream_t stream)
{
    if (!master_dev || !m_dev || !v_dev || !grad_dev || !params_dev || step < 1 || !(lr > 0) || !(beta1 >= 0) ||
        !(beta1 < 1) || !(beta2 >= 0) || !(beta2 < 1) || !(eps > 0))
        return TSDF_EINVAL;
    hipLaunchKernelGGL(adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream, master_dev, m_dev, v_dev,
                       grad_dev, (uint16_t *)params_dev, step, lr, beta1, beta2, eps);
    return hipGetLastError() == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

uint64_t tsdf_mlp_samples_workspace_bytes(int32_t width, int32_t height)
{
    const uint64_t nb = ((uint64_t)width * height + 255) / 256;
    return nb * 4 + nb * 8 + 8;
}

tsdf_status tsdf_mlp_collect_samples(const float *depth_dev, const float *feat_dev, const uint8_t *valid_dev,
                                     const float *vertex_dev, const tsdf_intrinsics *K, const double pose_c2w[12],
                                     void *workspace_dev, uint64_t *count_dev, int64_t cap, float *x_out_dev,
                                     float *r_out_dev, hipStream_t stream)
{
    if (!depth_dev || !feat_dev || !valid_dev || !vertex_dev || !K || !pose_c2w || !workspace_dev || !count_dev ||
        cap < 0 || (cap > 0 && (!x_out_dev || !r_out_dev)) || K->width <= 0 || K->height <= 0)
        return TSDF_EINVAL;
    Camera cam;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) cam.R[3 * r + c] = pose_c2w[4 * r + c];
        cam.t[r] = pose_c2w[4 * r + 3];
    }
    cam.fx = K->fx;
    cam.fy = K->fy;
    cam.cx = K->cx;
    cam.cy = K->cy;
    cam.width = K->width;
    cam.height = K->height;
    const int64_t n = (int64_t)K->width * K->height;
    const int nb = (int)((n + 255) / 256);
    uint32_t *counts = (uint32_t *)workspace_dev;
    uint64_t *base = (uint64_t *)((uint8_t *)workspace_dev + (((uint64_t)nb * 4 + 7) & ~7ull));
    hipLaunchKernelGGL(sample_count_kernel, dim3(nb), dim3(256), 0, stream, depth_dev, (const float4 *)feat_dev,
                       valid_dev, (const float4 *)vertex_dev, cam, n, counts);
    hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(64), 0, stream, counts, nb, base, count_dev);
    hipLaunchKernelGGL(sample_write_kernel, dim3(nb), dim3(256), 0, stream, depth_dev, (const float4 *)feat_dev,
                       valid_dev, (const float4 *)vertex_dev, cam, n, (const uint64_t *)base, cap,
                       (float4 *)x_out_dev, r_out_dev);
    return hipGetLastError() == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

}  // extern "C"

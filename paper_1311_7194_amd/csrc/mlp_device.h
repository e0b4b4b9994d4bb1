// Learned measurement-noise model: device building blocks (gfx950).
//
// The paper weights measurements by a variance that grows with the fourth
// power of depth and notes that edges are noisier (Section 1, Section 7.1).
// The learned model predicts log sigma^2 (m^2) per pixel with a 4-32-32-1
// perceptron (SiLU) from four features: depth, incidence cosine, distance to
// a depth discontinuity (capped at 16 px) and radial pixel distance / fx.
// Weights are bfloat16, accumulation float32; layer-1 and layer-2 inputs are
// rounded to bfloat16 (round to nearest even).  Layer 2 runs on the matrix
// cores (v_mfma_f32_32x32x16_bf16), one wavefront = 64 samples = two 32-row
// tiles.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsdf {

constexpr int kMlpIn = 4, kMlpHidden = 32;
constexpr int kMlpParams = 1249;      // W1[32][4] b1[32] W2[32][32] b2[32] W3[32] b3
constexpr int kMlpParamsPadded = 1256;
enum { MLP_W1 = 0, MLP_B1 = 128, MLP_W2 = 160, MLP_B2 = 1184, MLP_W3 = 1216, MLP_B3 = 1248 };
constexpr int kEdgeCap = 16;

typedef short i16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

// D += A B on the matrix cores, v_mfma_f32_32x32x16_bf16 (A 32x16, B 16x32,
// D 32x32, bf16 in, fp32 accumulate).  Lane l supplies A[l % 32][8 (l / 32) + e]
// and B[8 (l / 32) + e][l % 32] for e = 0..7 (bf16 bit patterns) and holds
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in accumulator r.
__device__ __forceinline__ f32x16_t mfma_bf16_k16(i16x8_t a, i16x8_t b, f32x16_t c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                    c, 0, 0, 0);
}

// bfloat16 round to nearest even, as the bit pattern and as a value: the
// hardware conversion, which for every finite input gives the bits of adding
// 0x7fff plus the kept lowest bit and truncating
__device__ __forceinline__ uint16_t bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ __forceinline__ float bf16_round(float f) { return __uint_as_float((uint32_t)bf16_bits(f) << 16); }
__device__ __forceinline__ float bf16_value(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// SiLU with the hardware reciprocal (one rounding more than a division; the
// result is rounded to bfloat16 next).  exp(-a) = inf for very negative a
// gives rcp(inf) = 0, the limit.
__device__ __forceinline__ float silu(float a) { return a * __builtin_amdgcn_rcpf(1.0f + __expf(-a)); }
__device__ __forceinline__ float silu_grad(float a)
{
    const float sg = __builtin_amdgcn_rcpf(1.0f + __expf(-a));
    return sg * (1.0f + a * (1.0f - sg));
}

// Parameters staged in LDS as floats (values of the bf16 weights).
struct MlpParamsLds {
    float p[kMlpParamsPadded];
};

__device__ __forceinline__ void mlp_stage_params(MlpParamsLds &s, const uint16_t *__restrict__ params, int tid,
                                                 int nthreads)
{
    // eight loads per thread in flight before their LDS stores (clamped
    // indices keep them in bounds)
    for (int k0 = tid; k0 < kMlpParams; k0 += 8 * nthreads) {
        uint16_t b[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) b[q] = params[min(k0 + q * nthreads, kMlpParams - 1)];
#pragma unroll
        for (int q = 0; q < 8; ++q)
            if (k0 + q * nthreads < kMlpParams) s.p[k0 + q * nthreads] = bf16_value(b[q]);
    }
}

// Per-wavefront LDS scratch for the layer-2 operands and the output reduction.
struct MlpWaveLds {
    uint16_t h1[64][kMlpHidden + 4];   // bf16 layer-1 activations per sample (padded rows)
    float t3[64][kMlpHidden + 1];      // per (sample, hidden unit) output-layer terms
};

// Layer 2 for the 64 samples of a wavefront on the matrix cores:
// acc[tile] = h1[32 tile rows][32] x W2^T[32][32] (bf16 in, fp32 out), two
// K = 16 steps per tile.
__device__ __forceinline__ void mlp_layer2_mfma(const MlpWaveLds &w, const uint16_t *__restrict__ W2bits, int lane,
                                                f32x16_t acc[2])
{
    const int col = lane & 31, kh = 8 * (lane >> 5);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x16_t c = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < kMlpHidden / 16; ++kk) {
            i16x8_t a, b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = (short)w.h1[32 * t + col][16 * kk + kh + e];
                // B[k][n] = W2[n][k]: output unit n = col, input k
                b[e] = (short)W2bits[col * kMlpHidden + 16 * kk + kh + e];
            }
            c = mfma_bf16_k16(a, b, c);
        }
        acc[t] = c;
    }
}

// Forward pass of the 64 samples held by one wavefront (one sample per lane;
// x are the raw features).  P: parameters (LDS floats), W2bits: W2 as bf16
// bits.  Returns log sigma^2 for the lane's sample; when a2out is non-null
// the layer-2 pre-activations are kept in the accumulator layout (for the
// backward pass).  Every thread of the workgroup must call it (it holds
// workgroup barriers).

__device__ __forceinline__ float mlp_forward_wave(const MlpParamsLds &P, const uint16_t *__restrict__ W2bits,
                                                  MlpWaveLds &w, const float x[4], int lane, float a2out[2][16])
{
    const float x0[4] = {bf16_round(x[0]), bf16_round(x[1]), bf16_round(x[2]), bf16_round(x[3])};
#pragma unroll
    for (int o = 0; o < kMlpHidden; ++o) {
        float a = P.p[MLP_B1 + o];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) a += P.p[MLP_W1 + o * kMlpIn + i] * x0[i];
        w.h1[lane][o] = bf16_bits(silu(a));
    }
    __syncthreads();
    f32x16_t acc[2];
    mlp_layer2_mfma(w, W2bits, lane, acc);
    const int col = lane & 31;
    const float b2 = P.p[MLP_B2 + col], w3 = P.p[MLP_W3 + col];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = 32 * t + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const float a2 = acc[t][r] + b2;
            if (a2out) a2out[t][r] = a2;
            w.t3[row][col] = w3 * bf16_round(silu(a2));
        }
    __syncthreads();
    float s = P.p[MLP_B3];
#pragma unroll
    for (int o = 0; o < kMlpHidden; ++o) s += w.t3[lane][o];
    return s;
}

// Inference-only forward pass with a small LDS footprint (the integration
// path runs it in every preparation workgroup, where LDS bounds occupancy):
// one bf16 activation tile per wavefront holds h1 for layer 2, then h2 for
// the output layer, which also runs on the matrix cores (W3 as the only
// non-zero column of B).  Same rounding points as mlp_forward_wave; only the
// order of the output layer's FP32 sum differs.
struct MlpInferLds {
    uint16_t h[64][kMlpHidden + 4];   // bf16 activations, one sample per row
    float out[64];
};

__device__ __forceinline__ float mlp_infer_wave(const MlpParamsLds &P, const uint16_t *__restrict__ params,
                                                MlpInferLds &w, const float x[4], int lane)
{
    const float x0[4] = {bf16_round(x[0]), bf16_round(x[1]), bf16_round(x[2]), bf16_round(x[3])};
#pragma unroll
    for (int o = 0; o < kMlpHidden; ++o) {
        float a = P.p[MLP_B1 + o];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) a += P.p[MLP_W1 + o * kMlpIn + i] * x0[i];
        w.h[lane][o] = bf16_bits(silu(a));
    }
    __syncthreads();
    const int col = lane & 31, kh = 8 * (lane >> 5), rh = 4 * (lane >> 5);
    f32x16_t acc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x16_t c = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < kMlpHidden / 16; ++kk) {
            i16x8_t a, b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = (short)w.h[32 * t + col][16 * kk + kh + e];
                b[e] = (short)params[MLP_W2 + col * kMlpHidden + 16 * kk + kh + e];
            }
            c = mfma_bf16_k16(a, b, c);
        }
        acc[t] = c;
    }
    __syncthreads();   // h1 has been read: the tile now takes h2
    const float b2 = P.p[MLP_B2 + col];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r)
            w.h[32 * t + 8 * (r >> 2) + rh + (r & 3)][col] = bf16_bits(silu(acc[t][r] + b2));
    __syncthreads();
    // s[m] = b3 + sum_o h2[m][o] W3[o]: M = samples, N = 1 (column 0 of B), K = o
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x16_t c = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < kMlpHidden / 16; ++kk) {
            i16x8_t a, b;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                a[e] = (short)w.h[32 * t + col][16 * kk + kh + e];
                b[e] = col == 0 ? (short)params[MLP_W3 + 16 * kk + kh + e] : (short)0;
            }
            c = mfma_bf16_k16(a, b, c);
        }
        if (col == 0) {
#pragma unroll
            for (int r = 0; r < 16; ++r) w.out[32 * t + 8 * (r >> 2) + rh + (r & 3)] = c[r] + P.p[MLP_B3];
        }
    }
    __syncthreads();
    return w.out[lane];
}

}  // namespace tsdf

// Point-to-plane ICP iteration on raycast maps (Section 6); tsdf_icp.h
// documents the steps.
//
//   icp_pairs_kernel  one pass over the live pixels: live point and normal,
//                     projective match into the model maps, rejection, and
//                     per-thread sums of the unscaled normal equations and the
//                     box of the kept points; workgroups write partial sums
//   icp_solve_kernel  one workgroup: adds the partials, forms the scaled
//                     system from the unscaled sums, eigen-decomposes it,
//                     keeps the directions above the threshold, and composes
//                     the pose
//
// Every step of the matching is evaluated in double precision without
// contractions, in a fixed operation order, so that which pixel a point
// matches and whether a pair is kept are decided exactly as the defined
// expressions decide them.
#include <math.h>

#include <hip/hip_runtime.h>

#include "tsdf_icp.h"

static_assert(sizeof(tsdf_icp_result) == 600 && sizeof(tsdf_icp_params) == 32, "ICP records in tsdf_icp.h");

namespace tsdf {
namespace {

constexpr int kIcpThreads = 256;
constexpr int kIcpMaxGroups = 1024;
constexpr int kSums = 29;      // 21 upper-triangle entries, 6 right-hand sides, e^2, pair count
constexpr int kVals = 35;      // + box minimum (3) and maximum (3)
constexpr int kStride = 36;    // doubles per partial

struct IcpArgs {
    double Rm[9], tm[3];       // model pose, camera to world
    double fx, fy, cx, cy;
    int32_t width, height;
    double dist2;              // dist_max^2
    double cos2;               // cos_min^2
    double theta;
    int32_t shrink;
};

__device__ __forceinline__ bool depth_ok(float d) { return d > 0.0f && isfinite(d); }

// Reduces the kVals values of every lane of the workgroup into lane 0 of
// wave 0: sums for the first kSums, minimum and maximum for the box.
__device__ __forceinline__ void block_reduce(double v[kVals], double (*lds)[kVals])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < kVals; ++k) {
            const double o = __shfl_xor(v[k], off);
            v[k] = k < kSums ? v[k] + o : (k < kSums + 3 ? fmin(v[k], o) : fmax(v[k], o));
        }
    }
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < kVals; ++k) lds[wave][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int w = 1; w < kIcpThreads / 64; ++w)
#pragma unroll
            for (int k = 0; k < kVals; ++k)
                v[k] = k < kSums ? v[k] + lds[w][k] : (k < kSums + 3 ? fmin(v[k], lds[w][k]) : fmax(v[k], lds[w][k]));
}

__device__ __forceinline__ void init_vals(double v[kVals])
{
#pragma unroll
    for (int k = 0; k < kVals; ++k) v[k] = k < kSums ? 0.0 : (k < kSums + 3 ? INFINITY : -INFINITY);
}

__global__ __launch_bounds__(kIcpThreads) void icp_pairs_kernel(const float *__restrict__ depth,
                                                                const float4 *__restrict__ mvert,
                                                                const float4 *__restrict__ mnorm,
                                                                const double *__restrict__ pose, IcpArgs a,
                                                                double *__restrict__ partial)
{
#pragma clang fp contract(off)
    __shared__ double lds[kIcpThreads / 64][kVals];
    const int W = a.width, H = a.height;
    double Rc[9], tc[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Rc[3 * r + c] = pose[4 * r + c];
        tc[r] = pose[4 * r + 3];
    }
    double v[kVals];
    init_vals(v);
    const long long npix = (long long)W * H;
    for (long long pix = (long long)blockIdx.x * kIcpThreads + threadIdx.x; pix < npix;
         pix += (long long)gridDim.x * kIcpThreads) {
        const int i = (int)(pix % W), j = (int)(pix / W);
        if (i + 1 >= W || j + 1 >= H) continue;
        const float d0 = depth[pix], dr = depth[pix + 1], dd = depth[pix + W];
        if (!(depth_ok(d0) && depth_ok(dr) && depth_ok(dd))) continue;
        // live point and its neighbours through the pixel centres, camera frame
        const double ui = ((double)i - a.cx) / a.fx, ui1 = ((double)(i + 1) - a.cx) / a.fx;
        const double vj = ((double)j - a.cy) / a.fy, vj1 = ((double)(j + 1) - a.cy) / a.fy;
        const double D0 = d0, Dr = dr, Dd = dd;
        const double x0[3] = {ui * D0, vj * D0, D0};
        const double right[3] = {ui1 * Dr - x0[0], vj * Dr - x0[1], Dr - x0[2]};
        const double down[3] = {ui * Dd - x0[0], vj1 * Dd - x0[1], Dd - x0[2]};
        const double nc[3] = {down[1] * right[2] - down[2] * right[1], down[2] * right[0] - down[0] * right[2],
                              down[0] * right[1] - down[1] * right[0]};
        double p[3], nw[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            p[r] = ((Rc[3 * r] * x0[0] + Rc[3 * r + 1] * x0[1]) + Rc[3 * r + 2] * x0[2]) + tc[r];
            nw[r] = (Rc[3 * r] * nc[0] + Rc[3 * r + 1] * nc[1]) + Rc[3 * r + 2] * nc[2];
        }
        // projective match in the model camera
        const double e0 = p[0] - a.tm[0], e1 = p[1] - a.tm[1], e2 = p[2] - a.tm[2];
        const double xm = (a.Rm[0] * e0 + a.Rm[3] * e1) + a.Rm[6] * e2;
        const double ym = (a.Rm[1] * e0 + a.Rm[4] * e1) + a.Rm[7] * e2;
        const double zm = (a.Rm[2] * e0 + a.Rm[5] * e1) + a.Rm[8] * e2;
        if (!(zm > 0.0)) continue;
        const double fu = floor(a.fx * xm / zm + a.cx + 0.5), fv = floor(a.fy * ym / zm + a.cy + 0.5);
        if (!(fu >= 0.0 && fu < (double)W && fv >= 0.0 && fv < (double)H)) continue;
        const long long m = (long long)fv * W + (long long)fu;
        const float4 V = mvert[m];
        if (!(V.w > 0.0f)) continue;
        const float4 N = mnorm[m];
        const double q[3] = {V.x, V.y, V.z}, n[3] = {N.x, N.y, N.z};
        // rejection: distance, then normal deviation
        const double dq[3] = {p[0] - q[0], p[1] - q[1], p[2] - q[2]};
        if (!((dq[0] * dq[0] + dq[1] * dq[1]) + dq[2] * dq[2] <= a.dist2)) continue;
        const double dot = (nw[0] * n[0] + nw[1] * n[1]) + nw[2] * n[2];
        const double nn = (nw[0] * nw[0] + nw[1] * nw[1]) + nw[2] * nw[2];
        const double mm = (n[0] * n[0] + n[1] * n[1]) + n[2] * n[2];
        if (!(dot > 0.0 && dot * dot >= a.cos2 * (nn * mm))) continue;
        // the pair's rows of the normal equations: g = (p x n, n), e = (p - q) . n
        const double g[6] = {p[1] * n[2] - p[2] * n[1], p[2] * n[0] - p[0] * n[2], p[0] * n[1] - p[1] * n[0],
                             n[0], n[1], n[2]};
        const double e = (dq[0] * n[0] + dq[1] * n[1]) + dq[2] * n[2];
        int k = 0;
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int c = r; c < 6; ++c) v[k++] += g[r] * g[c];
#pragma unroll
        for (int r = 0; r < 6; ++r) v[21 + r] += g[r] * e;
        v[27] += e * e;
        v[28] += 1.0;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            v[kSums + r] = fmin(v[kSums + r], fmin(p[r], q[r]));
            v[kSums + 3 + r] = fmax(v[kSums + 3 + r], fmax(p[r], q[r]));
        }
    }
    block_reduce(v, lds);
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < kVals; ++k) partial[(size_t)blockIdx.x * kStride + k] = v[k];
}

// Eigen-decomposition of the symmetric 6x6 matrix A (destroyed) by cyclic
// Jacobi rotations: A V = V diag(lam).
__device__ void jacobi6(double A[36], double V[36], double lam[6])
{
    for (int k = 0; k < 36; ++k) V[k] = (k % 7 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int r = 0; r < 6; ++r) {
            diag += A[7 * r] * A[7 * r];
            for (int c = r + 1; c < 6; ++c) off += A[6 * r + c] * A[6 * r + c];
        }
        if (!(off > 1e-36 * diag)) break;
        for (int p = 0; p < 5; ++p)
            for (int q = p + 1; q < 6; ++q) {
                const double apq = A[6 * p + q];
                if (apq == 0.0) continue;
                // rotation in the (p, q) plane that zeroes A[p][q]
                const double th = (A[7 * q] - A[7 * p]) / (2.0 * apq);
                const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 6; ++k) {   // A <- A J
                    const double akp = A[6 * k + p], akq = A[6 * k + q];
                    A[6 * k + p] = c * akp - s * akq;
                    A[6 * k + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 6; ++k) {   // A <- J^T A
                    const double apk = A[6 * p + k], aqk = A[6 * q + k];
                    A[6 * p + k] = c * apk - s * aqk;
                    A[6 * q + k] = s * apk + c * aqk;
                }
                A[6 * p + q] = A[6 * q + p] = 0.0;
                for (int k = 0; k < 6; ++k) {   // V <- V J
                    const double vkp = V[6 * k + p], vkq = V[6 * k + q];
                    V[6 * k + p] = c * vkp - s * vkq;
                    V[6 * k + q] = s * vkp + c * vkq;
                }
            }
    }
    for (int k = 0; k < 6; ++k) lam[k] = A[7 * k];
}

__global__ __launch_bounds__(kIcpThreads) void icp_solve_kernel(const double *__restrict__ partial, int groups,
                                                                const double *__restrict__ pose, IcpArgs a,
                                                                tsdf_icp_result *__restrict__ res)
{
    __shared__ double lds[kIcpThreads / 64][kVals];
    double v[kVals];
    init_vals(v);
    for (int g = threadIdx.x; g < groups; g += kIcpThreads) {
        const double *pg = partial + (size_t)g * kStride;
#pragma unroll
        for (int k = 0; k < kVals; ++k)
            v[k] = k < kSums ? v[k] + pg[k] : (k < kSums + 3 ? fmin(v[k], pg[k]) : fmax(v[k], pg[k]));
    }
    block_reduce(v, lds);
    if (threadIdx.x != 0) return;

    // unscaled system: blocks Acc = sum c c^T, Acn = sum c n^T, Ann = sum n n^T, and sum g e
    double A[36];
    int k = 0;
    for (int r = 0; r < 6; ++r)
        for (int c = r; c < 6; ++c) A[6 * r + c] = A[6 * c + r] = v[k++];
    double b[6];
    for (int r = 0; r < 6; ++r) b[r] = -v[21 + r];
    const double N = v[28];
    double m[3] = {0.0, 0.0, 0.0}, S[3] = {1.0, 1.0, 1.0};
    if (a.shrink && N > 0.0) {
        for (int r = 0; r < 3; ++r) {
            m[r] = 0.5 * (v[kSums + r] + v[kSums + 3 + r]);
            const double ext = v[kSums + 3 + r] - v[kSums + r];
            S[r] = ext > 0.0 ? ext : 1.0;
        }
        // c^ = S^-1 (c - M n) with M n = m x n: the scaled blocks are
        //   S^-1 (Acc - Acn M^T - M Acn^T + M Ann M^T) S^-1,  S^-1 (Acn - M Ann),  Ann
        // and the right-hand side -S^-1 (sum c e - M sum n e), -sum n e
        const double M[9] = {0.0, -m[2], m[1], m[2], 0.0, -m[0], -m[1], m[0], 0.0};
        double Acc[9], Acn[9], Ann[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                Acc[3 * r + c] = A[6 * r + c];
                Acn[3 * r + c] = A[6 * r + 3 + c];
                Ann[3 * r + c] = A[6 * (r + 3) + 3 + c];
            }
        double MAnn[9], AcnMt[9], Bcn[9], Bcc[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s1 = 0.0, s2 = 0.0;
                for (int l = 0; l < 3; ++l) {
                    s1 += M[3 * r + l] * Ann[3 * l + c];
                    s2 += Acn[3 * r + l] * M[3 * c + l];
                }
                MAnn[3 * r + c] = s1;
                AcnMt[3 * r + c] = s2;
            }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double mam = 0.0;
                for (int l = 0; l < 3; ++l) mam += MAnn[3 * r + l] * M[3 * c + l];   // M Ann M^T
                Bcc[3 * r + c] = (Acc[3 * r + c] - AcnMt[3 * r + c] - AcnMt[3 * c + r] + mam) / (S[r] * S[c]);
                Bcn[3 * r + c] = (Acn[3 * r + c] - MAnn[3 * r + c]) / S[r];
            }
        double bc[3];
        for (int r = 0; r < 3; ++r) {
            double mb = 0.0;
            for (int l = 0; l < 3; ++l) mb += M[3 * r + l] * v[24 + l];
            bc[r] = -(v[21 + r] - mb) / S[r];
        }
        for (int r = 0; r < 3; ++r) {
            b[r] = bc[r];
            for (int c = 0; c < 3; ++c) {
                A[6 * r + c] = Bcc[3 * r + c];
                A[6 * r + 3 + c] = Bcn[3 * r + c];
                A[6 * (3 + c) + r] = Bcn[3 * r + c];
            }
        }
    }
    for (int q = 0; q < 36; ++q) res->C[q] = A[q];
    for (int q = 0; q < 6; ++q) res->b[q] = b[q];
    for (int q = 0; q < 3; ++q) {
        res->m[q] = m[q];
        res->S[q] = S[q];
    }
    res->residual2 = v[27];
    res->pairs = (int64_t)N;

    double P[12];
    for (int q = 0; q < 12; ++q) P[q] = pose[q];
    double x[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, lam[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int kept = 0;
    if (N > 0.0) {
        double Vec[36];
        jacobi6(A, Vec, lam);
        double xh[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int e = 0; e < 6; ++e) {
            const bool keep = lam[e] > 0.0 && (a.theta >= 0.0 ? lam[e] / N > a.theta : true);
            if (!keep) continue;
            ++kept;
            double vb = 0.0;
            for (int r = 0; r < 6; ++r) vb += Vec[6 * r + e] * b[r];
            for (int r = 0; r < 6; ++r) xh[r] += Vec[6 * r + e] * (vb / lam[e]);
        }
        // back to the unscaled increment: r = S^-1 r^, t = t^ - r x m
        const double rr[3] = {xh[0] / S[0], xh[1] / S[1], xh[2] / S[2]};
        const double rxm[3] = {rr[1] * m[2] - rr[2] * m[1], rr[2] * m[0] - rr[0] * m[2], rr[0] * m[1] - rr[1] * m[0]};
        x[0] = rr[0];
        x[1] = rr[1];
        x[2] = rr[2];
        for (int q = 0; q < 3; ++q) x[3 + q] = xh[3 + q] - rxm[q];
        // R_inc = Rz(gamma) Ry(beta) Rx(alpha); pose' = R_inc pose + t_inc
        double sa, ca, sb, cb, sg, cg;
        sincos(x[0], &sa, &ca);
        sincos(x[1], &sb, &cb);
        sincos(x[2], &sg, &cg);
        const double Rx[9] = {1.0, 0.0, 0.0, 0.0, ca, -sa, 0.0, sa, ca};
        const double Ry[9] = {cb, 0.0, sb, 0.0, 1.0, 0.0, -sb, 0.0, cb};
        const double Rz[9] = {cg, -sg, 0.0, sg, cg, 0.0, 0.0, 0.0, 1.0};
        double Ryx[9], Ri[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int l = 0; l < 3; ++l) s += Ry[3 * r + l] * Rx[3 * l + c];
                Ryx[3 * r + c] = s;
            }
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s = 0.0;
                for (int l = 0; l < 3; ++l) s += Rz[3 * r + l] * Ryx[3 * l + c];
                Ri[3 * r + c] = s;
            }
        double Pn[12];
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 4; ++c) {
                double s = 0.0;
                for (int l = 0; l < 3; ++l) s += Ri[3 * r + l] * P[4 * l + c];
                Pn[4 * r + c] = s;
            }
            Pn[4 * r + 3] += x[3 + r];
        }
        for (int q = 0; q < 12; ++q) P[q] = Pn[q];
        // eigenvalues per pair, ascending
        for (int e = 0; e < 6; ++e) lam[e] /= N;
        for (int e = 1; e < 6; ++e)
            for (int f = e; f > 0 && lam[f - 1] > lam[f]; --f) {
                const double t = lam[f];
                lam[f] = lam[f - 1];
                lam[f - 1] = t;
            }
    }
    for (int q = 0; q < 12; ++q) res->pose[q] = P[q];
    for (int q = 0; q < 6; ++q) {
        res->x[q] = x[q];
        res->lambda[q] = lam[q];
    }
    res->kept = kept;
    res->pad = 0;
}

int icp_groups(int32_t width, int32_t height)
{
    const long long npix = (long long)width * height;
    const long long g = (npix + kIcpThreads - 1) / kIcpThreads;
    return (int)(g < kIcpMaxGroups ? g : kIcpMaxGroups);
}

bool icp_pose_ok(const double *p)
{
    for (int q = 0; q < 12; ++q)
        if (!isfinite(p[q])) return false;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            const double dot = p[4 * r] * p[4 * c] + p[4 * r + 1] * p[4 * c + 1] + p[4 * r + 2] * p[4 * c + 2];
            if (fabs(dot - (r == c ? 1.0 : 0.0)) > 1e-6) return false;
        }
    const double det = p[0] * (p[5] * p[10] - p[6] * p[9]) - p[1] * (p[4] * p[10] - p[6] * p[8]) +
                       p[2] * (p[4] * p[9] - p[5] * p[8]);
    return det > 0;
}

}  // namespace
}  // namespace tsdf

using namespace tsdf;

extern "C" {

uint64_t tsdf_icp_workspace_bytes(int32_t width, int32_t height)
{
    if (width < 1 || height < 1 || width > 16384 || height > 16384) return 0;
    return (uint64_t)icp_groups(width, height) * kStride * sizeof(double);
}

tsdf_status tsdf_icp_step(const float *depth_dev, const tsdf_intrinsics *K, const float *model_vertex_dev,
                          const float *model_normal_dev, const double model_pose_c2w[12], const double *pose_dev,
                          const tsdf_icp_params *params, void *workspace_dev, uint64_t workspace_bytes,
                          tsdf_icp_result *result_dev, hipStream_t stream)
{
    if (!depth_dev || !K || !model_vertex_dev || !model_normal_dev || !model_pose_c2w || !pose_dev || !params ||
        !workspace_dev || !result_dev)
        return TSDF_EINVAL;
    if (!(isfinite(K->fx) && isfinite(K->fy) && isfinite(K->cx) && isfinite(K->cy) && K->fx > 0 && K->fy > 0))
        return TSDF_EINVAL;
    const uint64_t need = tsdf_icp_workspace_bytes(K->width, K->height);
    if (need == 0 || workspace_bytes < need) return TSDF_EINVAL;
    if (!icp_pose_ok(model_pose_c2w)) return TSDF_EINVAL;
    if (!(isfinite(params->dist_max) && params->dist_max > 0) ||
        !(isfinite(params->cos_min) && params->cos_min >= -1.0 && params->cos_min <= 1.0) ||
        !isfinite(params->theta) || (params->shrink != 0 && params->shrink != 1))
        return TSDF_EINVAL;
    IcpArgs a;
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) a.Rm[3 * r + c] = model_pose_c2w[4 * r + c];
        a.tm[r] = model_pose_c2w[4 * r + 3];
    }
    a.fx = K->fx;
    a.fy = K->fy;
    a.cx = K->cx;
    a.cy = K->cy;
    a.width = K->width;
    a.height = K->height;
    a.dist2 = params->dist_max * params->dist_max;
    a.cos2 = params->cos_min * params->cos_min;
    a.theta = params->theta;
    a.shrink = params->shrink;
    const int groups = icp_groups(K->width, K->height);
    double *partial = (double *)workspace_dev;
    hipLaunchKernelGGL(icp_pairs_kernel, dim3(groups), dim3(kIcpThreads), 0, stream, depth_dev,
                       (const float4 *)model_vertex_dev, (const float4 *)model_normal_dev, pose_dev, a, partial);
    hipLaunchKernelGGL(icp_solve_kernel, dim3(1), dim3(kIcpThreads), 0, stream, partial, groups, pose_dev, a,
                       result_dev);
    return hipGetLastError() == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

}  // extern "C"

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

#include <mutex>

#include <hip/hip_runtime.h>

#include "tsdf_icp.h"

static_assert(sizeof(tsdf_icp_result) == 600 && sizeof(tsdf_icp_params) == 32, "ICP records in tsdf_icp.h");

namespace tsdf {
namespace {

constexpr int kIcpThreads = 256;
constexpr int kIcpMaxGroups = 512;
// Per-workgroup partials, stored value-major ([kPartial][groups]):
//   0..20 upper triangle of sum g g^T, g = (p x n, n); 21..26 sum g e;
//   27 sum e^2; 28 pair count; 29..31 zero;
//   32..34 -min and 35..37 max of the kept p and q per axis; 38, 39 unused.
constexpr int kPartial = 40;

struct IcpArgs {
    double Rm[9], tm[3];       // model pose, camera to world
    double fx, fy, cx, cy;
    int32_t width, height;
    double dist2;              // dist_max^2
    double cos2;               // cos_min^2
    double theta;
    int32_t shrink;
    double P0[12];             // current pose when the kernels get no device pose
};

// The current pose estimate: the device record or, for a chain's first
// iteration, the host pose passed in the kernel arguments.
__device__ __forceinline__ double pose_at(const double *pose, const IcpArgs &a, int q)
{
    return pose ? pose[q] : a.P0[q];
}

__device__ __forceinline__ bool depth_ok(float d) { return d > 0.0f && isfinite(d); }

struct ReduceLds {
    double s[kIcpThreads / 64][32];
    double x[kIcpThreads / 64][8];
    double tot[kPartial];
};

// Workgroup reduction of 32 sums and 8 maxima per lane into L.tot (visible
// to every thread on return).  Within a wavefront, recursive halving: at
// each exchange a lane keeps one half of its values and sends the other, so
// the sums take 32 exchanges instead of 6 per value.  Afterwards lanes 2m and
// 2m + 1 hold the wavefront's total of sum m, and lanes 8m..8m + 7 its
// maximum m.
__device__ __forceinline__ void block_reduce(const double s[32], const double x[8], ReduceLds &L)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
    double h16[16], h8[8], h4[4], h2[2];
#pragma unroll
    for (int k = 0; k < 16; ++k) h16[k] = (b5 ? s[k + 16] : s[k]) + __shfl_xor(b5 ? s[k] : s[k + 16], 32);
#pragma unroll
    for (int k = 0; k < 8; ++k) h8[k] = (b4 ? h16[k + 8] : h16[k]) + __shfl_xor(b4 ? h16[k] : h16[k + 8], 16);
#pragma unroll
    for (int k = 0; k < 4; ++k) h4[k] = (b3 ? h8[k + 4] : h8[k]) + __shfl_xor(b3 ? h8[k] : h8[k + 4], 8);
#pragma unroll
    for (int k = 0; k < 2; ++k) h2[k] = (b2 ? h4[k + 2] : h4[k]) + __shfl_xor(b2 ? h4[k] : h4[k + 2], 4);
    double h1 = (b1 ? h2[1] : h2[0]) + __shfl_xor(b1 ? h2[0] : h2[1], 2);
    h1 += __shfl_xor(h1, 1);
    if (!(lane & 1)) L.s[wave][lane >> 1] = h1;
    double g4[4], g2[2];
#pragma unroll
    for (int k = 0; k < 4; ++k) g4[k] = fmax(b5 ? x[k + 4] : x[k], __shfl_xor(b5 ? x[k] : x[k + 4], 32));
#pragma unroll
    for (int k = 0; k < 2; ++k) g2[k] = fmax(b4 ? g4[k + 2] : g4[k], __shfl_xor(b4 ? g4[k] : g4[k + 2], 16));
    double g1 = fmax(b3 ? g2[1] : g2[0], __shfl_xor(b3 ? g2[0] : g2[1], 8));
    g1 = fmax(g1, __shfl_xor(g1, 4));
    g1 = fmax(g1, __shfl_xor(g1, 2));
    g1 = fmax(g1, __shfl_xor(g1, 1));
    if (!(lane & 7)) L.x[wave][lane >> 3] = g1;
    __syncthreads();
    const int t = threadIdx.x;
    if (t < 32)
        L.tot[t] = (L.s[0][t] + L.s[1][t]) + (L.s[2][t] + L.s[3][t]);
    else if (t < kPartial)
        L.tot[t] = fmax(fmax(L.x[0][t - 32], L.x[1][t - 32]), fmax(L.x[2][t - 32], L.x[3][t - 32]));
    __syncthreads();
}

__device__ __forceinline__ void init_acc(double s[32], double x[8])
{
#pragma unroll
    for (int k = 0; k < 32; ++k) s[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = -INFINITY;
}

__global__ __launch_bounds__(kIcpThreads) void icp_pairs_kernel(const float *__restrict__ depth,
                                                                const float4 *__restrict__ mvert,
                                                                const float4 *__restrict__ mnorm,
                                                                const double *__restrict__ pose, IcpArgs a,
                                                                double *__restrict__ partial)
{
#pragma clang fp contract(off)
    __shared__ ReduceLds L;
    const int W = a.width, H = a.height;
    double Rc[9], tc[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) Rc[3 * r + c] = pose_at(pose, a, 4 * r + c);
        tc[r] = pose_at(pose, a, 4 * r + 3);
    }
    double v[32], bx[8];
    init_acc(v, bx);
    const uint32_t npix = (uint32_t)W * (uint32_t)H;   // at most 16384^2 < 2^32
    for (uint32_t pix = blockIdx.x * kIcpThreads + threadIdx.x; pix < npix; pix += gridDim.x * kIcpThreads) {
        const int j = (int)(pix / (uint32_t)W), i = (int)(pix - (uint32_t)j * (uint32_t)W);
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
            bx[r] = fmax(bx[r], fmax(-p[r], -q[r]));
            bx[3 + r] = fmax(bx[3 + r], fmax(p[r], q[r]));
        }
    }
    block_reduce(v, bx, L);
    if (threadIdx.x < kPartial) partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = L.tot[threadIdx.x];
}

// Parallel cyclic Jacobi for a symmetric 6x6 matrix on one wavefront.  Lane
// l < 36 holds element (l / 6, l % 6) of A and of the eigenvector matrix V.
// A sweep is five rounds of three disjoint plane rotations: in round k the
// index x5 = 3k mod 5 pairs with 5 and the others as (x5 + 1, x5 + 4) and
// (x5 + 2, x5 + 3) mod 5 (indices x, y < 5 pair when x + y = k mod 5), which
// covers all 15 pairs.  Disjoint rotations commute and do not touch each
// other's 2x2 blocks, so a round applies its three at once: A <- J^T A J,
// V <- V J.  The pivots are read out of their lanes as wave-uniform values
// and every lane computes the three rotations itself.
__device__ __forceinline__ double lane_value(double x, int lane)
{
    const unsigned long long u = __double_as_longlong(x);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)u, lane);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(u >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Reciprocal and reciprocal square root to about an ulp: the hardware
// estimate and two Newton steps.  The rotations only have to (nearly) zero
// their pivot and stay orthogonal, which c = 1/sqrt(1 + t^2), s = t c does
// to rounding whatever the accuracy of t.
__device__ __forceinline__ double fast_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double fast_rsqrt(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y * fma(-0.5 * x * y, y, 1.5);
}

__device__ __forceinline__ void plane_rotation(double app, double aqq, double apq, double &c, double &s)
{
    if (apq == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    const double th = 0.5 * (aqq - app) * fast_rcp(apq);
    const double at = fabs(th);
    // t = sign(th) / (|th| + sqrt(th^2 + 1)), with sqrt(h) = h / sqrt(h);
    // beyond |th| = 1e100 (where th^2 would overflow) t = 1 / (2 |th|) to rounding
    const double h = at < 1e100 ? fma(at, at, 1.0) : 1.0;
    const double den = at < 1e100 ? at + h * fast_rsqrt(h) : 2.0 * at;
    const double t = (th >= 0.0 ? 1.0 : -1.0) * fast_rcp(den);
    c = fast_rsqrt(fma(t, t, 1.0));
    s = t * c;
}

// Called by the 64 lanes of one wavefront; sA and sV0 (read) and sV, sLam
// (written) in LDS.  sV0 is the rotation the sweeps start from: null for the
// identity, or an orthogonal V0 when sA holds V0^T A V0, so that the
// eigenvectors come out for A itself.
__device__ void jacobi6_wave(const double *sA, const double *sV0, double *sV, double *sLam)
{
    const int lane = threadIdx.x & 63;
    const bool own = lane < 36;
    const int r = own ? lane / 6 : 0, c = own ? lane % 6 : 0;
    double a = own ? sA[lane] : 0.0;
    double v = own ? (sV0 ? sV0[lane] : (r == c ? 1.0 : 0.0)) : 0.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int p = 0; p < 6; ++p) {
            const double d = lane_value(a, 7 * p);
            diag += d * d;
            for (int q = p + 1; q < 6; ++q) {
                const double o = lane_value(a, 6 * p + q);
                off += o * o;
            }
        }
        if (!(off > 1e-26 * diag)) break;   // off-diagonal norm below 1e-13 of the diagonal's
        for (int k = 0; k < 5; ++k) {
            const int x5 = (3 * k) % 5;
            int P[3], Q[3];
            P[0] = x5;
            Q[0] = 5;
            P[1] = min((x5 + 1) % 5, (x5 + 4) % 5);
            Q[1] = max((x5 + 1) % 5, (x5 + 4) % 5);
            P[2] = min((x5 + 2) % 5, (x5 + 3) % 5);
            Q[2] = max((x5 + 2) % 5, (x5 + 3) % 5);
            double cs[3], sn[3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                plane_rotation(lane_value(a, 7 * P[i]), lane_value(a, 7 * Q[i]), lane_value(a, 6 * P[i] + Q[i]), cs[i],
                               sn[i]);
            // this lane's row and column: pair, partner, and column of J
            // (J[x][x] = cos, J[partner][x] = -sin for the pair's smaller index, +sin otherwise)
            const int ir = (r == P[0] || r == Q[0]) ? 0 : ((r == P[1] || r == Q[1]) ? 1 : 2);
            const int ic = (c == P[0] || c == Q[0]) ? 0 : ((c == P[1] || c == Q[1]) ? 1 : 2);
            const int pr = ir == 0 ? P[0] : (ir == 1 ? P[1] : P[2]), qr = ir == 0 ? Q[0] : (ir == 1 ? Q[1] : Q[2]);
            const int pc = ic == 0 ? P[0] : (ic == 1 ? P[1] : P[2]), qc = ic == 0 ? Q[0] : (ic == 1 ? Q[1] : Q[2]);
            const int r2 = r == pr ? qr : pr, c2 = c == pc ? qc : pc;
            const double cr = ir == 0 ? cs[0] : (ir == 1 ? cs[1] : cs[2]);
            const double cc = ic == 0 ? cs[0] : (ic == 1 ? cs[1] : cs[2]);
            const double snr = ir == 0 ? sn[0] : (ir == 1 ? sn[1] : sn[2]);
            const double snc = ic == 0 ? sn[0] : (ic == 1 ? sn[1] : sn[2]);
            const double sr = r == pr ? -snr : snr, sc = c == pc ? -snc : snc;
            const double a_rc2 = __shfl(a, 6 * r + c2), a_r2c = __shfl(a, 6 * r2 + c), a_r2c2 = __shfl(a, 6 * r2 + c2);
            const double v_rc2 = __shfl(v, 6 * r + c2);
            const double an = (cr * cc * a + cr * sc * a_rc2) + (sr * cc * a_r2c + sr * sc * a_r2c2);
            a = c == r2 ? 0.0 : an;   // the rotated pair's off-diagonal entries
            v = v * cc + v_rc2 * sc;
        }
    }
    if (own) {
        sV[lane] = v;
        if (r == c) sLam[r] = a;
    }
}

// The system solved in this iteration (scaled when shrink is set).
struct IcpSystem {
    double A[36], b[6], m[3], S[3];
    double N, e2;
};

// From the reduced sums: the unscaled blocks Acc = sum c c^T, Acn = sum c n^T,
// Ann = sum n n^T and sum g e; with shrink, the scaled system by the change
// of variables c^ = S^-1 (c - M n), M n = m x n:
//   S^-1 (Acc - Acn M^T - M Acn^T + M Ann M^T) S^-1,  S^-1 (Acn - M Ann),  Ann,
//   right-hand side -S^-1 (sum c e - M sum n e), -sum n e.
__device__ void system_of(const double *v, const IcpArgs &a, IcpSystem &sys)
{
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
            const double lo = -v[32 + r], hi = v[35 + r];
            m[r] = 0.5 * (lo + hi);
            const double ext = hi - lo;
            S[r] = ext > 0.0 ? ext : 1.0;
        }
        const double M[9] = {0.0, -m[2], m[1], m[2], 0.0, -m[0], -m[1], m[0], 0.0};
        double MAnn[9], AcnMt[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double s1 = 0.0, s2 = 0.0;
                for (int l = 0; l < 3; ++l) {
                    s1 += M[3 * r + l] * A[6 * (l + 3) + 3 + c];    // M Ann
                    s2 += A[6 * r + 3 + l] * M[3 * c + l];          // Acn M^T
                }
                MAnn[3 * r + c] = s1;
                AcnMt[3 * r + c] = s2;
            }
        double Bcc[9], Bcn[9], bc[3];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double mam = 0.0;
                for (int l = 0; l < 3; ++l) mam += MAnn[3 * r + l] * M[3 * c + l];   // M Ann M^T
                Bcc[3 * r + c] = (A[6 * r + c] - AcnMt[3 * r + c] - AcnMt[3 * c + r] + mam) / (S[r] * S[c]);
                Bcn[3 * r + c] = (A[6 * r + 3 + c] - MAnn[3 * r + c]) / S[r];
            }
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
    for (int q = 0; q < 36; ++q) sys.A[q] = A[q];
    for (int q = 0; q < 6; ++q) sys.b[q] = b[q];
    for (int q = 0; q < 3; ++q) {
        sys.m[q] = m[q];
        sys.S[q] = S[q];
    }
    sys.N = N;
    sys.e2 = v[27];
}

// Thresholded solution from the eigen-decomposition (V columns, lam), back-
// substitution, and the pose update; writes the result record.
__device__ void solve_and_update(const IcpSystem &sys, const double *V, const double *lam_in, const IcpArgs &a,
                                 const double *pose, tsdf_icp_result *res)
{
    const double N = sys.N;
    for (int q = 0; q < 36; ++q) res->C[q] = sys.A[q];
    for (int q = 0; q < 6; ++q) res->b[q] = sys.b[q];
    for (int q = 0; q < 3; ++q) {
        res->m[q] = sys.m[q];
        res->S[q] = sys.S[q];
    }
    res->residual2 = sys.e2;
    res->pairs = (int64_t)N;
    double P[12];
    for (int q = 0; q < 12; ++q) P[q] = pose_at(pose, a, q);
    double x[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, lam[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int kept = 0;
    if (N > 0.0) {
        for (int e = 0; e < 6; ++e) lam[e] = lam_in[e];
        double xh[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int e = 0; e < 6; ++e) {
            const bool keep = lam[e] > 0.0 && (a.theta >= 0.0 ? lam[e] / N > a.theta : true);
            if (!keep) continue;
            ++kept;
            double vb = 0.0;
            for (int r = 0; r < 6; ++r) vb += V[6 * r + e] * sys.b[r];
            for (int r = 0; r < 6; ++r) xh[r] += V[6 * r + e] * (vb / lam[e]);
        }
        // back to the unscaled increment: r = S^-1 r^, t = t^ - r x m
        const double *S = sys.S, *m = sys.m;
        const double rr[3] = {xh[0] / S[0], xh[1] / S[1], xh[2] / S[2]};
        const double rxm[3] = {rr[1] * m[2] - rr[2] * m[1], rr[2] * m[0] - rr[0] * m[2], rr[0] * m[1] - rr[1] * m[0]};
        for (int q = 0; q < 3; ++q) {
            x[q] = rr[q];
            x[3 + q] = xh[3 + q] - rxm[q];
        }
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

// warm: start the eigen-decomposition from the previous iteration's
// eigenvectors (kept in vwork): the system changes little from one iteration
// to the next, so V^T A V is nearly diagonal and a sweep or two finish it.
__global__ __launch_bounds__(kIcpThreads) void icp_solve_kernel(const double *__restrict__ partial, int groups,
                                                                const double *__restrict__ pose, IcpArgs a,
                                                                tsdf_icp_result *__restrict__ res,
                                                                double *__restrict__ vwork, int warm)
{
    __shared__ ReduceLds L;
    __shared__ IcpSystem sys;
    __shared__ double sV[36], sLam[6], sV0[36], sB[36], sA2[36];
    const int t = threadIdx.x;
    if (warm && t < 36) sV0[t] = vwork[t];
    double v[32], bx[8];
    init_acc(v, bx);
#pragma unroll 4
    for (int g = threadIdx.x; g < groups; g += kIcpThreads) {
#pragma unroll
        for (int k = 0; k < 32; ++k) v[k] += partial[(size_t)k * groups + g];
#pragma unroll
        for (int k = 0; k < 8; ++k) bx[k] = fmax(bx[k], partial[(size_t)(32 + k) * groups + g]);
    }
    block_reduce(v, bx, L);
    if (t == 0) system_of(L.tot, a, sys);
    __syncthreads();
    const bool use_warm = warm && sys.N > 0.0;
    if (use_warm) {   // sB = (V0^T A V0), symmetrised
        const int r = t / 6, c = t % 6;
        if (t < 36) {
            double s = 0.0;
            for (int l = 0; l < 6; ++l) s += sys.A[6 * r + l] * sV0[6 * l + c];
            sB[t] = s;
        }
        __syncthreads();
        if (t < 36) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += sV0[6 * k + r] * sB[6 * k + c];
            sA2[t] = s;
        }
        __syncthreads();
        if (t < 36) sB[t] = 0.5 * (sA2[t] + sA2[6 * c + r]);
        __syncthreads();
    }
    if (t < 64 && sys.N > 0.0) jacobi6_wave(use_warm ? sB : sys.A, use_warm ? sV0 : nullptr, sV, sLam);
    __syncthreads();
    if (t < 36) vwork[t] = sys.N > 0.0 ? sV[t] : (t % 7 == 0 ? 1.0 : 0.0);
    if (t == 0) solve_and_update(sys, sV, sLam, a, pose, res);
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

// Scratch memory of tsdf_icp_run_noalloc: the per-workgroup partial sums of
// at most kIcpMaxGroups workgroups (the cap of icp_groups, whatever the frame
// size) followed by the 36 warm-start eigenvector entries, the layout the
// caller's workspace has in tsdf_icp_run.  Each device holds its own copy
// from the first call on it until the process ends.
constexpr int kScratchDoubles = kIcpMaxGroups * kPartial + 36;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices];

// Device address of the current device's `scratch` (in host code the name
// stands for a host-side shadow, never for device memory); looked up once
// per device with that device current.  nullptr on failure.
double *scratch_address()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch_ptr[dev] = (double *)ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace tsdf

using namespace tsdf;

extern "C" {

uint64_t tsdf_icp_workspace_bytes(int32_t width, int32_t height)
{
    if (width < 1 || height < 1 || width > 16384 || height > 16384) return 0;
    // partials, then the last eigenvectors (36 doubles) for a warm start
    return (uint64_t)icp_groups(width, height) * kPartial * sizeof(double) + 36 * sizeof(double);
}

}  // extern "C"

namespace {

// Validates the arguments shared by the ICP entry points (all but the
// workspace) and fills the kernel arguments.
tsdf_status icp_args(const float *depth_dev, const tsdf_intrinsics *K, const float *model_vertex_dev,
                     const float *model_normal_dev, const double *model_pose_c2w, const tsdf_icp_params *params,
                     const void *result_dev, IcpArgs &a)
{
    if (!depth_dev || !K || !model_vertex_dev || !model_normal_dev || !model_pose_c2w || !params || !result_dev)
        return TSDF_EINVAL;
    if (!(isfinite(K->fx) && isfinite(K->fy) && isfinite(K->cx) && isfinite(K->cy) && K->fx > 0 && K->fy > 0))
        return TSDF_EINVAL;
    if (tsdf_icp_workspace_bytes(K->width, K->height) == 0) return TSDF_EINVAL;
    if (!icp_pose_ok(model_pose_c2w)) return TSDF_EINVAL;
    if (!(isfinite(params->dist_max) && params->dist_max > 0) ||
        !(isfinite(params->cos_min) && params->cos_min >= -1.0 && params->cos_min <= 1.0) ||
        !isfinite(params->theta) || (params->shrink != 0 && params->shrink != 1))
        return TSDF_EINVAL;
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
    for (int q = 0; q < 12; ++q) a.P0[q] = 0.0;
    return TSDF_OK;
}

void icp_enqueue(const float *depth_dev, const float *mv, const float *mn, const double *pose_dev, const IcpArgs &a,
                 void *workspace_dev, tsdf_icp_result *result_dev, int warm, hipStream_t stream)
{
    const int groups = icp_groups(a.width, a.height);
    double *partial = (double *)workspace_dev;
    double *vwork = partial + (size_t)groups * kPartial;
    hipLaunchKernelGGL(icp_pairs_kernel, dim3(groups), dim3(kIcpThreads), 0, stream, depth_dev, (const float4 *)mv,
                       (const float4 *)mn, pose_dev, a, partial);
    hipLaunchKernelGGL(icp_solve_kernel, dim3(1), dim3(kIcpThreads), 0, stream, partial, groups, pose_dev, a,
                       result_dev, vwork, warm);
}

}  // namespace

extern "C" {

tsdf_status tsdf_icp_step(const float *depth_dev, const tsdf_intrinsics *K, const float *model_vertex_dev,
                          const float *model_normal_dev, const double model_pose_c2w[12], const double *pose_dev,
                          const tsdf_icp_params *params, void *workspace_dev, uint64_t workspace_bytes,
                          tsdf_icp_result *result_dev, hipStream_t stream)
{
    IcpArgs a;
    if (!pose_dev) return TSDF_EINVAL;
    const tsdf_status st = icp_args(depth_dev, K, model_vertex_dev, model_normal_dev, model_pose_c2w, params,
                                    result_dev, a);
    if (st != TSDF_OK) return st;
    if (!workspace_dev || workspace_bytes < tsdf_icp_workspace_bytes(K->width, K->height)) return TSDF_EINVAL;
    icp_enqueue(depth_dev, model_vertex_dev, model_normal_dev, pose_dev, a, workspace_dev, result_dev, 0, stream);
    return hipGetLastError() == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

}  // extern "C"

namespace {

// Validates the arguments of a chain of iterations (all but the workspace).
tsdf_status icp_run_args(const float *depth_dev, const tsdf_intrinsics *K, const float *model_vertex_dev,
                         const float *model_normal_dev, const double *model_pose_c2w, const double *pose_init_c2w,
                         const tsdf_icp_params *params, int32_t iters, const void *results_dev, IcpArgs &a)
{
    if (!pose_init_c2w || iters < 1 || iters > 1024 || !icp_pose_ok(pose_init_c2w)) return TSDF_EINVAL;
    const tsdf_status st = icp_args(depth_dev, K, model_vertex_dev, model_normal_dev, model_pose_c2w, params,
                                    results_dev, a);
    if (st != TSDF_OK) return st;
    for (int q = 0; q < 12; ++q) a.P0[q] = pose_init_c2w[q];
    return TSDF_OK;
}

tsdf_status icp_run_enqueue(const float *depth_dev, const float *mv, const float *mn, const IcpArgs &a, int32_t iters,
                            void *workspace_dev, tsdf_icp_result *results_dev, hipStream_t stream)
{
    for (int k = 0; k < iters; ++k)
        icp_enqueue(depth_dev, mv, mn, k == 0 ? nullptr : results_dev[k - 1].pose, a, workspace_dev, results_dev + k,
                    k > 0, stream);
    return hipGetLastError() == hipSuccess ? TSDF_OK : TSDF_EHIP;
}

}  // namespace

extern "C" {

tsdf_status tsdf_icp_run(const float *depth_dev, const tsdf_intrinsics *K, const float *model_vertex_dev,
                         const float *model_normal_dev, const double model_pose_c2w[12],
                         const double pose_init_c2w[12], const tsdf_icp_params *params, int32_t iters,
                         void *workspace_dev, uint64_t workspace_bytes, tsdf_icp_result *results_dev,
                         hipStream_t stream)
{
    IcpArgs a;
    const tsdf_status st = icp_run_args(depth_dev, K, model_vertex_dev, model_normal_dev, model_pose_c2w,
                                        pose_init_c2w, params, iters, results_dev, a);
    if (st != TSDF_OK) return st;
    if (!workspace_dev || workspace_bytes < tsdf_icp_workspace_bytes(K->width, K->height)) return TSDF_EINVAL;
    return icp_run_enqueue(depth_dev, model_vertex_dev, model_normal_dev, a, iters, workspace_dev, results_dev,
                           stream);
}

tsdf_status tsdf_icp_run_noalloc(const float *depth_dev, const tsdf_intrinsics *K, const float *model_vertex_dev,
                                 const float *model_normal_dev, const double model_pose_c2w[12],
                                 const double pose_init_c2w[12], const tsdf_icp_params *params, int32_t iters,
                                 tsdf_icp_result *results_dev, hipStream_t stream)
{
    IcpArgs a;
    const tsdf_status st = icp_run_args(depth_dev, K, model_vertex_dev, model_normal_dev, model_pose_c2w,
                                        pose_init_c2w, params, iters, results_dev, a);
    if (st != TSDF_OK) return st;
    // the frame-size check above bounds the workgroups at kIcpMaxGroups, so
    // the partials always fit; checked again against the array itself
    if (tsdf_icp_workspace_bytes(K->width, K->height) > sizeof(double) * (uint64_t)kScratchDoubles)
        return TSDF_EINVAL;
    double *ws = scratch_address();
    if (!ws) return TSDF_EHIP;
    return icp_run_enqueue(depth_dev, model_vertex_dev, model_normal_dev, a, iters, ws, results_dev, stream);
}

}  // extern "C"

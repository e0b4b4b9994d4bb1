/*
 * Oracle of the learned measurement-noise model — TEST INFRASTRUCTURE ONLY.
 *
 * The paper models the measurement variance p_k as growing with the fourth
 * power of depth and notes that edge measurements are noisier (Section 1,
 * Section 7.1).  The learned model predicts log sigma^2 per pixel from four
 * features with a 4-32-32-1 perceptron (SiLU), trained by Gaussian negative
 * log-likelihood on residuals of the fused surface.  This file restates, in
 * double precision with bfloat16 rounding at the defined points:
 *   - the per-pixel features,
 *   - the forward pass, the loss and its analytic gradients,
 * so that the HIP kernels can be checked against it.  Build with
 * -ffp-contract=off.
 *
 * Rounding points (bf16 = round to nearest even of the value's float32):
 *   x0 = bf16(features); a1 = W1 x0 + b1; h1 = bf16(silu(a1));
 *   a2 = W2 h1 + b2; h2 = bf16(silu(a2)); s = W3 . h2 + b3.
 *   Backward: ds = (1 - r^2 exp(-s)) / 2; the layer-2 products use
 *   e2 = bf16(da2) (dW2 = e2 h1^T, dh1 = W2^T e2); everything else unrounded.
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NI 4
#define NH 32
#define NPARAM (NH * NI + NH + NH * NH + NH + NH + 1)

/* Parameter layout (shared with the packed device format):
 *   W1[32][4], b1[32], W2[32][32], b2[32], W3[32], b3  (1249 values) */
enum { OFF_W1 = 0, OFF_B1 = 128, OFF_W2 = 160, OFF_B2 = 1184, OFF_W3 = 1216, OFF_B3 = 1248 };

int orc_mlp_param_count(void) { return NPARAM; }

/* bfloat16 round-to-nearest-even of the float32 nearest to x. */
double orc_bf16(double x)
{
    float f = (float)x;
    uint32_t b;
    memcpy(&b, &f, 4);
    if ((b & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf/nan unchanged */
    uint32_t lsb = (b >> 16) & 1u;
    b += 0x7fffu + lsb;
    b &= 0xffff0000u;
    memcpy(&f, &b, 4);
    return (double)f;
}

static double silu(double a) { return a / (1.0 + exp(-a)); }
static double silu_grad(double a)
{
    double sg = 1.0 / (1.0 + exp(-a));
    return sg * (1.0 + a * (1.0 - sg));
}

/*
 * Per-pixel features from a depth map [H][W] (metres, <= 0 invalid):
 *   f0 = D
 *   f1 = |cos| of the angle between the view ray and the surface normal; the
 *        normal is the cross product of the central differences of the
 *        back-projected points along i and j (all four neighbours valid)
 *   f2 = min(Euclidean pixel distance to the nearest discontinuity, 16) / 16;
 *        a discontinuity is a valid pixel with a 4-neighbour that is invalid
 *        or differs by more than 5 % of its depth (neighbours outside the
 *        image do not count); pixels outside the image are not discontinuities
 *   f3 = sqrt((i - cx)^2 + (j - cy)^2) / fx
 * valid[k] = 1 when all features exist (D valid and the normal defined).
 */
void orc_mlp_features(const float *depth, int32_t W, int32_t H, const double K[4], double *feat, int32_t *valid)
{
    const double fx = K[0], fy = K[1], cx = K[2], cy = K[3];
    int64_t n = (int64_t)W * H;
    /* discontinuity map */
    unsigned char *disc = (unsigned char *)malloc((size_t)n);
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            int64_t k = (int64_t)j * W + i;
            float D = depth[k];
            disc[k] = 0;
            if (!(D > 0.0f) || !isfinite(D)) continue;
            const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
            for (int q = 0; q < 4; ++q) {
                int ii = i + di[q], jj = j + dj[q];
                if (ii < 0 || jj < 0 || ii >= W || jj >= H) continue;
                float Dn = depth[(int64_t)jj * W + ii];
                if (!(Dn > 0.0f) || !isfinite(Dn) || fabs((double)Dn - (double)D) > 0.05 * (double)D) disc[k] = 1;
            }
        }
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            int64_t k = (int64_t)j * W + i;
            double *f = feat + 4 * k;
            float D = depth[k];
            valid[k] = 0;
            f[0] = f[1] = f[2] = f[3] = 0.0;
            if (!(D > 0.0f) || !isfinite(D)) continue;
            f[0] = D;
            f[3] = sqrt((i - cx) * (i - cx) + (j - cy) * (j - cy)) / fx;
            /* nearest discontinuity within the 16-pixel cap (brute force) */
            double best = 16.0;
            for (int dj = -16; dj <= 16; ++dj)
                for (int di = -16; di <= 16; ++di) {
                    int ii = i + di, jj = j + dj;
                    if (ii < 0 || jj < 0 || ii >= W || jj >= H) continue;
                    if (!disc[(int64_t)jj * W + ii]) continue;
                    double dist = sqrt((double)(di * di + dj * dj));
                    if (dist < best) best = dist;
                }
            f[2] = best / 16.0;
            if (i < 1 || j < 1 || i >= W - 1 || j >= H - 1) continue;
            float Dl = depth[k - 1], Dr = depth[k + 1], Du = depth[k - W], Dd = depth[k + W];
            if (!(Dl > 0.0f && Dr > 0.0f && Du > 0.0f && Dd > 0.0f)) continue;
            double pl[3] = {(i - 1 - cx) / fx * Dl, (j - cy) / fy * Dl, Dl};
            double pr[3] = {(i + 1 - cx) / fx * Dr, (j - cy) / fy * Dr, Dr};
            double pu[3] = {(i - cx) / fx * Du, (j - 1 - cy) / fy * Du, Du};
            double pd[3] = {(i - cx) / fx * Dd, (j + 1 - cy) / fy * Dd, Dd};
            double a[3] = {pr[0] - pl[0], pr[1] - pl[1], pr[2] - pl[2]};
            double b[3] = {pd[0] - pu[0], pd[1] - pu[1], pd[2] - pu[2]};
            double nrm[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
            double nl = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
            double ray[3] = {(i - cx) / fx, (j - cy) / fy, 1.0};
            double rl = sqrt(ray[0] * ray[0] + ray[1] * ray[1] + 1.0);
            if (!(nl > 0.0)) continue;
            f[1] = fabs(nrm[0] * ray[0] + nrm[1] * ray[1] + nrm[2] * ray[2]) / (nl * rl);
            valid[k] = 1;
        }
    free(disc);
}

/* Forward pass for n samples; x is n*4 features, params 1249 values (taken
 * as bf16 values: the caller passes bf16-representable numbers); out s[n]. */
void orc_mlp_forward(const double *params, const double *x, int64_t n, double *s)
{
    const double *W1 = params + OFF_W1, *b1 = params + OFF_B1, *W2 = params + OFF_W2, *b2 = params + OFF_B2,
                 *W3 = params + OFF_W3, b3 = params[OFF_B3];
    for (int64_t k = 0; k < n; ++k) {
        double x0[NI], h1[NH], h2[NH];
        for (int i = 0; i < NI; ++i) x0[i] = orc_bf16(x[4 * k + i]);
        for (int o = 0; o < NH; ++o) {
            double a = b1[o];
            for (int i = 0; i < NI; ++i) a += W1[o * NI + i] * x0[i];
            h1[o] = orc_bf16(silu(a));
        }
        for (int o = 0; o < NH; ++o) {
            double a = b2[o];
            for (int i = 0; i < NH; ++i) a += W2[o * NH + i] * h1[i];
            h2[o] = orc_bf16(silu(a));
        }
        double out = b3;
        for (int i = 0; i < NH; ++i) out += W3[i] * h2[i];
        s[k] = out;
    }
}

/* Mean Gaussian negative log-likelihood 0.5 (s + r^2 exp(-s)) over n samples
 * and its gradient with respect to the 1249 parameters (grad: summed over
 * samples, divided by n).  Returns the mean loss.  If round_bf16 is 0 every
 * bf16 rounding is skipped (smooth function, for finite differences). */
double orc_mlp_loss_grad(const double *params, const double *x, const double *r, int64_t n, double *grad,
                         int32_t round_bf16)
{
    const double *W1 = params + OFF_W1, *b1 = params + OFF_B1, *W2 = params + OFF_W2, *b2 = params + OFF_B2,
                 *W3 = params + OFF_W3, b3 = params[OFF_B3];
#define RND(v) (round_bf16 ? orc_bf16(v) : (v))
    for (int p = 0; p < NPARAM; ++p) grad[p] = 0.0;
    double loss = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double x0[NI], a1[NH], h1[NH], a2[NH], h2[NH];
        for (int i = 0; i < NI; ++i) x0[i] = RND(x[4 * k + i]);
        for (int o = 0; o < NH; ++o) {
            double a = b1[o];
            for (int i = 0; i < NI; ++i) a += W1[o * NI + i] * x0[i];
            a1[o] = a;
            h1[o] = RND(silu(a));
        }
        for (int o = 0; o < NH; ++o) {
            double a = b2[o];
            for (int i = 0; i < NH; ++i) a += W2[o * NH + i] * h1[i];
            a2[o] = a;
            h2[o] = RND(silu(a));
        }
        double s = b3;
        for (int i = 0; i < NH; ++i) s += W3[i] * h2[i];
        double e = exp(-s);
        loss += 0.5 * (s + r[k] * r[k] * e);
        double ds = 0.5 * (1.0 - r[k] * r[k] * e);
        /* output layer */
        grad[OFF_B3] += ds;
        double da2[NH], e2[NH];
        for (int i = 0; i < NH; ++i) {
            grad[OFF_W3 + i] += ds * h2[i];
            da2[i] = ds * W3[i] * silu_grad(a2[i]);
            e2[i] = RND(da2[i]);
        }
        /* layer 2 */
        double dh1[NH];
        for (int i = 0; i < NH; ++i) dh1[i] = 0.0;
        for (int o = 0; o < NH; ++o) {
            grad[OFF_B2 + o] += da2[o];
            for (int i = 0; i < NH; ++i) {
                grad[OFF_W2 + o * NH + i] += e2[o] * h1[i];
                dh1[i] += W2[o * NH + i] * e2[o];
            }
        }
        /* layer 1 */
        for (int o = 0; o < NH; ++o) {
            double da1 = dh1[o] * silu_grad(a1[o]);
            grad[OFF_B1 + o] += da1;
            for (int i = 0; i < NI; ++i) grad[OFF_W1 + o * NI + i] += da1 * x0[i];
        }
    }
#undef RND
    for (int p = 0; p < NPARAM; ++p) grad[p] /= (double)n;
    return loss / (double)n;
}

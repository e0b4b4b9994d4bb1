/*
 * CPU oracle for sparse TSDF fusion and raycasting — TEST INFRASTRUCTURE ONLY.
 * Plain double precision, no blocking or fusion beyond what the method
 * states.  Build with -ffp-contract=off so that every expression below is
 * evaluated as written (no fused multiply-add).
 *
 * Paper passages followed:
 *   Eq. (1)               truncated signed distance with sentinel chi
 *   Section 4, Fig. 4-5   blocks of M^3 voxels, dense offset table, -1 = empty
 *   Fig. 4 caption        a block is allocated when anything but chi is stored in it
 *   Section 7.1 (end)     projective measurement T_k: project, distance to the depth sample
 *   Algorithm 1, 2, 3     the plain, weighted and Kalman updates
 *   Section 5             raycast of the sparse field into depth and normal maps
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define BLOCK 8
#define BVOX 512
#define CHI 2.0

struct orc_volume {
    int32_t G[3];        /* voxels per axis */
    int32_t N[3];        /* blocks per axis */
    double vs;           /* voxel edge, metres */
    double origin[3];    /* min corner of the grid */
    double delta;        /* truncation distance, metres */
    double q_hat;        /* process variance Q / delta^2 */
    int32_t rule;        /* ORC_RULE_*: which update algorithm fuses measurements */
    int32_t weight_kind; /* ORC_WEIGHT_*: w_k of Algorithms 1 and 2 */
    double w, w_max;     /* constant weight; cap of the weight sum (Algorithm 2) */
    int32_t threads;     /* integration threads (1: the plain serial loop) */
    int32_t *offset;     /* N0*N1*N2 entries: block index or -1 */
    int32_t *keys;       /* cap*3 block coordinates, allocation order */
    double *T, *P;       /* cap*512 each */
    int64_t n_blocks, cap;
};

typedef struct {
    double R[3][3], t[3];
    double fx, fy, cx, cy;
    int32_t W, H;
} camera;

static int is_chi(double T) { return fabs(T) > 1.0; }

static void load_camera(camera *c, const double K[4], const double pose[12], int32_t W, int32_t H)
{
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) c->R[r][k] = pose[4 * r + k];
        c->t[r] = pose[4 * r + 3];
    }
    c->fx = K[0];
    c->fy = K[1];
    c->cx = K[2];
    c->cy = K[3];
    c->W = W;
    c->H = H;
}

orc_volume *orc_create(const int32_t dims[3], double voxel_size, const double origin[3],
                       double trunc_voxels, double q_hat, int64_t capacity_blocks)
{
    for (int a = 0; a < 3; ++a)
        if (dims[a] <= 0 || dims[a] % BLOCK != 0) return NULL;
    if (!(voxel_size > 0) || !(trunc_voxels > 0) || capacity_blocks <= 0) return NULL;
    orc_volume *v = (orc_volume *)calloc(1, sizeof(orc_volume));
    int64_t nb = 1;
    for (int a = 0; a < 3; ++a) {
        v->G[a] = dims[a];
        v->N[a] = dims[a] / BLOCK;
        v->origin[a] = origin[a];
        nb *= v->N[a];
    }
    v->vs = voxel_size;
    v->delta = trunc_voxels * voxel_size;
    v->q_hat = q_hat;
    v->rule = ORC_RULE_KALMAN;
    v->weight_kind = ORC_WEIGHT_CONSTANT;
    v->w = 1.0;
    v->w_max = INFINITY;
    v->threads = 1;
    v->cap = capacity_blocks;
    v->offset = (int32_t *)malloc(sizeof(int32_t) * nb);
    for (int64_t b = 0; b < nb; ++b) v->offset[b] = -1;
    v->keys = (int32_t *)malloc(sizeof(int32_t) * 3 * capacity_blocks);
    v->T = (double *)malloc(sizeof(double) * BVOX * capacity_blocks);
    v->P = (double *)malloc(sizeof(double) * BVOX * capacity_blocks);
    if (!v->offset || !v->keys || !v->T || !v->P) {
        orc_destroy(v);
        return NULL;
    }
    return v;
}

void orc_destroy(orc_volume *v)
{
    if (!v) return;
    free(v->offset);
    free(v->keys);
    free(v->T);
    free(v->P);
    free(v);
}

int64_t orc_block_count(const orc_volume *v) { return v->n_blocks; }

static int64_t table_index(const orc_volume *v, int bx, int by, int bz)
{
    return ((int64_t)bz * v->N[1] + by) * v->N[0] + bx;
}

/* Offset-table lookup, then allocation from the store when absent (the
 * paper's free list reduces to "next unused block" here). Returns -1 when the
 * store is full.  With several integration threads (orc_set_threads) the
 * lookup reads the table entry atomically and an absent block is allocated
 * inside a critical section, which initialises it before publishing its
 * offset. */
static int64_t block_of(orc_volume *v, int bx, int by, int bz, int allocate, int64_t *new_blocks)
{
    int64_t ti = table_index(v, bx, by, bz);
    int32_t off;
#pragma omp atomic read seq_cst
    off = v->offset[ti];
    if (off >= 0 || !allocate) return off;
    int64_t b = -1;
#pragma omp critical(orc_allocate)
    {
        b = v->offset[ti];
        if (b < 0 && v->n_blocks < v->cap) {
            b = v->n_blocks++;
            v->keys[3 * b + 0] = bx;
            v->keys[3 * b + 1] = by;
            v->keys[3 * b + 2] = bz;
            for (int k = 0; k < BVOX; ++k) {
                v->T[b * BVOX + k] = CHI;
                v->P[b * BVOX + k] = 0.0;
            }
#pragma omp atomic write seq_cst
            v->offset[ti] = (int32_t)b;
            if (new_blocks) ++*new_blocks;
        }
    }
    return b;
}

/* Voxel centre x(g) = origin + (g + 0.5) * vs. */
static double voxel_centre(const orc_volume *v, int a, int g)
{
    return v->origin[a] + ((double)g + 0.5) * v->vs;
}

/*
 * The projective measurement of voxel g (Section 7.1, last paragraph, with
 * the signed distance of Eq. (1)):
 *   x_c = R^T (x - t); the voxel projects to the pixel whose centre is
 *   nearest, i = floor(fx x_c / z_c + cx + 0.5) and likewise j; the
 *   measurement is the camera-z distance s = D(i,j) - z_c, positive in front
 *   of the measured surface; it is chi when there is no depth sample or
 *   |s| > delta.
 * The expression order below is part of the definition: the decisions
 * (pixel index, |s| <= delta) are those of these exact double operations.
 * Returns 1 with (i, j, s) when the measurement is not chi.
 */
static int measure(const orc_volume *v, const camera *c, const float *depth, int gx, int gy, int gz,
                   int *pi, int *pj, double *ps, int *tie)
{
    double px = voxel_centre(v, 0, gx);
    double py = voxel_centre(v, 1, gy);
    double pz = voxel_centre(v, 2, gz);
    double dx = px - c->t[0];
    double dy = py - c->t[1];
    double dz = pz - c->t[2];
    double xc = c->R[0][0] * dx + c->R[1][0] * dy + c->R[2][0] * dz;
    double yc = c->R[0][1] * dx + c->R[1][1] * dy + c->R[2][1] * dz;
    double zc = c->R[0][2] * dx + c->R[1][2] * dy + c->R[2][2] * dz;
    if (!(zc > 0.0)) return 0;
    double u = c->fx * xc / zc + c->cx;
    double w = c->fy * yc / zc + c->cy;
    double fu = floor(u + 0.5);
    double fw = floor(w + 0.5);
    if (!(fu >= 0.0 && fu < (double)c->W && fw >= 0.0 && fw < (double)c->H)) return 0;
    int i = (int)fu, j = (int)fw;
    float D = depth[(int64_t)j * c->W + i];
    if (!(D > 0.0f) || !isfinite(D)) return 0;
    double s = (double)D - zc;
    if (tie) {
        double mu = fmin(u + 0.5 - fu, fu + 1.0 - (u + 0.5));
        double mw = fmin(w + 0.5 - fw, fw + 1.0 - (w + 0.5));
        double ms = fabs(fabs(s) - v->delta) / v->delta;
        *tie = (mu < 1e-9) || (mw < 1e-9) || (ms < 1e-9);
    }
    if (!(fabs(s) <= v->delta)) return 0;
    *pi = i;
    *pj = j;
    *ps = s;
    return 1;
}

/* Update algorithm of the volume's later integrations (see oracle.h). */
int orc_set_rule(orc_volume *v, int32_t rule, int32_t weight_kind, double w, double w_max)
{
    if (!v || rule < ORC_RULE_KALMAN || rule > ORC_RULE_WEIGHTED) return ORC_EINVAL;
    if (weight_kind != ORC_WEIGHT_CONSTANT && weight_kind != ORC_WEIGHT_INV_VARIANCE) return ORC_EINVAL;
    if (rule == ORC_RULE_RUNNING && (weight_kind != ORC_WEIGHT_CONSTANT || !(w > 0.0 && w <= 1.0))) return ORC_EINVAL;
    if (rule == ORC_RULE_WEIGHTED && weight_kind == ORC_WEIGHT_CONSTANT && !(w > 0.0 && isfinite(w)))
        return ORC_EINVAL;
    if (rule == ORC_RULE_WEIGHTED && !(w_max > 0.0)) return ORC_EINVAL;
    v->rule = rule;
    v->weight_kind = weight_kind;
    v->w = w;
    v->w_max = w_max;
    return ORC_OK;
}

/*
 * The three update rules of Section 7.1 (Algorithms 1, 2 and 3), in
 * normalised units.  All three move a voxel that already holds a value
 * toward the measurement by a gain g in [0, 1],
 *     T <- T + g (T_k - T),
 * and differ only in g and in the second per-voxel quantity S they carry:
 *   - Algorithm 1: g = w, a constant; S is not used.
 *   - Algorithm 2: S is the weight sum W of Eq. (10).  The weighted mean
 *     (W T + w_k T_k) / (W + w_k) is the increment with g = w_k / (W + w_k);
 *     afterwards W becomes min(W + w_k, W_max).
 *   - Algorithm 3: S is the variance P.  The prediction adds the process
 *     variance, P' = P + Q; g is the Kalman gain P' / (P' + p_k) and the
 *     variance becomes (1 - g) P'.
 * A voxel without a value (chi) takes the measurement itself; S starts at
 * the measurement's weight (Algorithm 2) or variance (Algorithm 3), with no
 * prediction added.  A value that leaves [-1, 1] is chi again.  A chi
 * measurement changes nothing.
 */
static void fuse_measurement(int rule, double *T, double *S, double Tk, double u, double q, double w_max)
{
    /* u: the constant weight w (Algorithm 1), the measurement's weight w_k
     * (Algorithm 2) or its variance p_k (Algorithm 3) */
    if (is_chi(Tk)) return;
    if (is_chi(*T)) {
        *T = Tk;
        if (rule != ORC_RULE_RUNNING) *S = u;
    } else {
        double g;
        if (rule == ORC_RULE_RUNNING) {
            g = u;
        } else if (rule == ORC_RULE_WEIGHTED) {
            g = u / (*S + u);
            *S = fmin(*S + u, w_max);
        } else {
            double pred = *S + q;
            g = pred / (pred + u);
            *S = (1.0 - g) * pred;
        }
        *T = *T + g * (Tk - *T);
    }
    if (is_chi(*T)) *T = CHI;
}

void orc_alg1_step(double *T, double Tk, double w)
{
    fuse_measurement(ORC_RULE_RUNNING, T, NULL, Tk, w, 0.0, 0.0);
}

void orc_alg2_step(double *T, double *Wsum, double Tk, double w, double w_max)
{
    fuse_measurement(ORC_RULE_WEIGHTED, T, Wsum, Tk, w, 0.0, w_max);
}

void orc_alg3_step(double *T, double *P, double Tk, double pk, double q)
{
    fuse_measurement(ORC_RULE_KALMAN, T, P, Tk, pk, q, 0.0);
}

/* Measurement variance in delta^2 units from the measured depth D.  The
 * paper: deviation grows quadratically with distance, so the variance grows
 * with its fourth power (Section 7.1, Kalman paragraph). */
static double measurement_variance(const orc_volume *v, int kind, double coeff, const double *phat_px,
                                   int64_t pix, double D)
{
    if (kind == ORC_NOISE_CONSTANT) return coeff;
    if (kind == ORC_NOISE_PER_PIXEL) return phat_px[pix];
    double sigma = coeff * D * D;
    return (sigma * sigma) / (v->delta * v->delta);
}

/*
 * Axis-aligned world box of the frustum cell of pixel (i, j) over camera
 * depths [z0, z1]: every point that projects to the pixel (by the nearest
 * centre rule) with depth in that range lies inside.  Used only to enumerate
 * candidate voxels; the measurement itself decides validity.
 */
static void cell_box(const camera *c, int i, int j, double z0, double z1, double lo[3], double hi[3])
{
    for (int a = 0; a < 3; ++a) {
        lo[a] = INFINITY;
        hi[a] = -INFINITY;
    }
    for (int k = 0; k < 8; ++k) {
        double u = i + ((k & 1) ? 0.5 : -0.5);
        double w = j + ((k & 2) ? 0.5 : -0.5);
        double z = (k & 4) ? z1 : z0;
        double xcam[3] = {(u - c->cx) / c->fx * z, (w - c->cy) / c->fy * z, z};
        for (int a = 0; a < 3; ++a) {
            double xw = c->R[a][0] * xcam[0] + c->R[a][1] * xcam[1] + c->R[a][2] * xcam[2] + c->t[a];
            if (xw < lo[a]) lo[a] = xw;
            if (xw > hi[a]) hi[a] = xw;
        }
    }
}

/*
 * The measurements of pixel (i, j): every voxel whose measurement is not chi
 * projects to exactly one pixel and lies in that pixel's frustum cell over
 * [D - delta, D + delta]; scanning the cell and keeping only the voxels that
 * project back to (i, j) visits each such voxel exactly once over the frame.
 * Returns ORC_EFULL when the block store runs out.
 */
static int integrate_pixel(orc_volume *v, const camera *c, const float *depth, int i, int j, int32_t noise_kind,
                           double coeff, const double *phat_px, orc_stats *s)
{
    const int32_t W = c->W;
    const double pad = 1e-3 * v->vs;
    float D = depth[(int64_t)j * W + i];
    if (!(D > 0.0f) || !isfinite(D)) return ORC_OK;
    double z0 = fmax((double)D - v->delta, 0.0), z1 = (double)D + v->delta;
    double lo[3], hi[3];
    int g0[3], g1[3];
    cell_box(c, i, j, z0, z1, lo, hi);
    for (int a = 0; a < 3; ++a) {
        double a0 = ceil((lo[a] - pad - v->origin[a]) / v->vs - 0.5);
        double a1 = floor((hi[a] + pad - v->origin[a]) / v->vs - 0.5);
        if (a0 < 0) a0 = 0;
        if (a1 > v->G[a] - 1) a1 = v->G[a] - 1;
        if (a0 > a1) return ORC_OK;
        g0[a] = (int)a0;
        g1[a] = (int)a1;
    }
    double pk = measurement_variance(v, noise_kind, coeff, phat_px, (int64_t)j * W + i, (double)D);
    /* Algorithm 2 keeps its weight sum W in P's place */
    double u = pk;
    if (v->rule == ORC_RULE_RUNNING)
        u = v->w;
    else if (v->rule == ORC_RULE_WEIGHTED)
        u = v->weight_kind == ORC_WEIGHT_INV_VARIANCE ? 1.0 / pk : v->w;
    for (int gz = g0[2]; gz <= g1[2]; ++gz)
        for (int gy = g0[1]; gy <= g1[1]; ++gy)
            for (int gx = g0[0]; gx <= g1[0]; ++gx) {
                int pi, pj, tie = 0;
                double sd;
                s->visited++;
                if (!measure(v, c, depth, gx, gy, gz, &pi, &pj, &sd, &tie)) continue;
                if (pi != i || pj != j) continue;
                if (tie) s->ties++;
                int64_t b = block_of(v, gx / BLOCK, gy / BLOCK, gz / BLOCK, 1, &s->new_blocks);
                if (b < 0) return ORC_EFULL;
                int64_t k = b * BVOX + (gx % BLOCK) + BLOCK * (gy % BLOCK) + BLOCK * BLOCK * (gz % BLOCK);
                fuse_measurement(v->rule, &v->T[k], &v->P[k], sd / v->delta, u, v->q_hat, v->w_max);
                s->updates++;
            }
    return ORC_OK;
}

int orc_set_threads(orc_volume *v, int32_t n_threads)
{
    if (!v || n_threads < 1) return ORC_EINVAL;
    v->threads = n_threads;
    return ORC_OK;
}

int orc_integrate(orc_volume *v, const float *depth, int32_t W, int32_t H, const double K[4],
                  const double pose[12], int32_t noise_kind, double coeff, const double *phat_px,
                  orc_stats *st)
{
    if (!v || !depth || W <= 0 || H <= 0) return ORC_EINVAL;
    if (noise_kind == ORC_NOISE_PER_PIXEL && !phat_px) return ORC_EINVAL;
    camera c;
    load_camera(&c, K, pose, W, H);
    orc_stats s = {0, 0, 0, 0};
    int status = ORC_OK;
    if (v->threads <= 1) {
        for (int j = 0; j < H && status == ORC_OK; ++j)
            for (int i = 0; i < W && status == ORC_OK; ++i)
                status = integrate_pixel(v, &c, depth, i, j, noise_kind, coeff, phat_px, &s);
    } else {
        /* each voxel belongs to one pixel, so rows of pixels update disjoint
         * voxels; only the block store is shared */
        int64_t upd = 0, nb = 0, ties = 0, vis = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(v->threads) reduction(+ : upd, nb, ties, vis)
        for (int j = 0; j < H; ++j) {
            orc_stats r = {0, 0, 0, 0};
            int full;
#pragma omp atomic read
            full = status;
            for (int i = 0; i < W && full == ORC_OK; ++i)
                if (integrate_pixel(v, &c, depth, i, j, noise_kind, coeff, phat_px, &r) != ORC_OK) {
                    full = ORC_EFULL;
#pragma omp atomic write
                    status = ORC_EFULL;
                }
            upd += r.updates;
            nb += r.new_blocks;
            ties += r.ties;
            vis += r.visited;
        }
        s.updates = upd;
        s.new_blocks = nb;
        s.ties = ties;
        s.visited = vis;
    }
    if (st) *st = s;
    return status;
}

/* ------------------------------------------------------------------ raycast */

/* Trilinear interpolation F of the stored distance over the 8 voxel centres
 * around p; invalid (returns 0) when any of them lies outside the grid, in
 * an empty block, or holds chi. */
int orc_sample(const orc_volume *v, const double p[3], double *F)
{
    int c[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
        double q = (p[a] - v->origin[a]) / v->vs - 0.5;
        double fl = floor(q);
        if (!(fl >= 0.0 && fl + 1.0 <= (double)(v->G[a] - 1))) return 0;
        c[a] = (int)fl;
        f[a] = q - fl;
    }
    double val[8];
    for (int k = 0; k < 8; ++k) {
        int g[3] = {c[0] + (k & 1), c[1] + ((k >> 1) & 1), c[2] + ((k >> 2) & 1)};
        int32_t b = v->offset[table_index(v, g[0] / BLOCK, g[1] / BLOCK, g[2] / BLOCK)];
        if (b < 0) return 0;
        double T = v->T[(int64_t)b * BVOX + (g[0] % BLOCK) + BLOCK * (g[1] % BLOCK) +
                        BLOCK * BLOCK * (g[2] % BLOCK)];
        if (is_chi(T)) return 0;
        val[k] = T;
    }
    double x00 = val[0] * (1.0 - f[0]) + val[1] * f[0];
    double x10 = val[2] * (1.0 - f[0]) + val[3] * f[0];
    double x01 = val[4] * (1.0 - f[0]) + val[5] * f[0];
    double x11 = val[6] * (1.0 - f[0]) + val[7] * f[0];
    double y0 = x00 * (1.0 - f[1]) + x10 * f[1];
    double y1 = x01 * (1.0 - f[1]) + x11 * f[1];
    *F = y0 * (1.0 - f[2]) + y1 * f[2];
    return 1;
}

static int sample_at(const orc_volume *v, const camera *c, const double d[3], double s, double *F)
{
    double p[3] = {c->t[0] + s * d[0], c->t[1] + s * d[1], c->t[2] + s * d[2]};
    return orc_sample(v, p, F);
}

/*
 * One ray (Section 5): march the lattice s_n = n * vs / 2 (n >= 1), take the
 * first n where F(s_n) > 0 >= F(s_{n+1}) with both valid (a front-facing
 * zero crossing), refine by bisection to 1e-9 voxel, and take the normal from
 * central differences of F one voxel apart along the world axes.
 */
static void cast_ray(const orc_volume *v, const camera *c, int i, int j, double *vert, double *nrm,
                     int32_t *flag)
{
    for (int k = 0; k < 4; ++k) vert[k] = nrm[k] = 0.0;
    *flag = 0;
    double dc[3] = {(i - c->cx) / c->fx, (j - c->cy) / c->fy, 1.0};
    double len = sqrt(dc[0] * dc[0] + dc[1] * dc[1] + dc[2] * dc[2]);
    double d[3];
    for (int a = 0; a < 3; ++a)
        d[a] = (c->R[a][0] * dc[0] + c->R[a][1] * dc[1] + c->R[a][2] * dc[2]) / len;
    /* samples can only be valid where every stencil voxel is inside the grid */
    double s_in = 0.0, s_out = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double lo = v->origin[a] + 0.5 * v->vs, hi = v->origin[a] + (v->G[a] - 0.5) * v->vs;
        if (d[a] == 0.0) {
            if (c->t[a] < lo || c->t[a] > hi) return;
            continue;
        }
        double s0 = (lo - c->t[a]) / d[a], s1 = (hi - c->t[a]) / d[a];
        if (s0 > s1) {
            double tmp = s0;
            s0 = s1;
            s1 = tmp;
        }
        if (s0 > s_in) s_in = s0;
        if (s1 < s_out) s_out = s1;
    }
    if (!(s_in <= s_out)) return;
    const double h = 0.5 * v->vs;
    int64_t n0 = (int64_t)ceil(s_in / h) - 1, n1 = (int64_t)floor(s_out / h) + 1;
    if (n0 < 1) n0 = 1;
    double Fprev = 0.0;
    int vprev = 0;
    for (int64_t n = n0; n <= n1; ++n) {
        double F;
        int valid = sample_at(v, c, d, (double)n * h, &F);
        if (valid && vprev && Fprev > 0.0 && F <= 0.0) {
            double lo = (double)(n - 1) * h, hi = (double)n * h;
            if (fabs(Fprev) < 1e-5 || fabs(F) < 1e-5) *flag |= ORC_MARGINAL;
            /* more than one root in the bracket makes the result ambiguous */
            int changes = 0, sub_invalid = 0, prev_pos = 1;
            for (int k = 1; k <= 64; ++k) {
                double Fk;
                if (!sample_at(v, c, d, lo + (hi - lo) * k / 64.0, &Fk)) {
                    sub_invalid = 1;
                    continue;
                }
                int pos = Fk > 0.0;
                if (pos != prev_pos) changes++;
                prev_pos = pos;
            }
            if (changes > 1 || sub_invalid) *flag |= ORC_AMBIGUOUS;
            while (hi - lo > 1e-9 * v->vs) {
                double mid = 0.5 * (lo + hi), Fm;
                if (!sample_at(v, c, d, mid, &Fm)) {
                    *flag |= ORC_BISECT_INVALID;
                    break;
                }
                if (Fm > 0.0)
                    lo = mid;
                else
                    hi = mid;
            }
            double s = 0.5 * (lo + hi);
            double p[3] = {c->t[0] + s * d[0], c->t[1] + s * d[1], c->t[2] + s * d[2]};
            double g[3];
            for (int a = 0; a < 3; ++a) {
                double pp[3] = {p[0], p[1], p[2]}, pm[3] = {p[0], p[1], p[2]};
                double Fp, Fm;
                pp[a] += v->vs;
                pm[a] -= v->vs;
                if (!orc_sample(v, pp, &Fp) || !orc_sample(v, pm, &Fm)) return;
                g[a] = Fp - Fm;
            }
            double gl = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            if (!(gl > 0.0)) return;
            for (int a = 0; a < 3; ++a) {
                vert[a] = p[a];
                nrm[a] = g[a] / gl;
            }
            vert[3] = nrm[3] = 1.0;
            *flag |= ORC_HIT;
            return;
        }
        Fprev = F;
        vprev = valid;
    }
}

int orc_raycast(const orc_volume *v, int32_t W, int32_t H, const double K[4], const double pose[12],
                const int32_t *pixels, int64_t n, double *vertex, double *normal, int32_t *flags,
                int32_t n_threads)
{
    if (!v || W <= 0 || H <= 0 || !vertex || !normal || !flags) return ORC_EINVAL;
    camera c;
    load_camera(&c, K, pose, W, H);
    int64_t count = pixels ? n : (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 64) num_threads(n_threads > 0 ? n_threads : 1)
    for (int64_t k = 0; k < count; ++k) {
        int i = pixels ? pixels[2 * k] : (int)(k % W);
        int j = pixels ? pixels[2 * k + 1] : (int)(k / W);
        cast_ray(v, &c, i, j, vertex + 4 * k, normal + 4 * k, flags + k);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------ import/export */

int64_t orc_export(const orc_volume *v, int32_t *keys, double *T, double *P, int64_t cap)
{
    int64_t n = v->n_blocks < cap ? v->n_blocks : cap;
    if (keys) memcpy(keys, v->keys, sizeof(int32_t) * 3 * n);
    if (T) memcpy(T, v->T, sizeof(double) * BVOX * n);
    if (P) memcpy(P, v->P, sizeof(double) * BVOX * n);
    return v->n_blocks;
}

/* Eviction (future work in Section 8: stream out the blocks that leave the
 * working volume): every block whose coordinates lie outside [lo, hi]
 * (inclusive, per axis) is copied out, in allocation order, and removed;
 * the remaining blocks keep their order and the offset table is rebuilt.
 * Returns the number of blocks evicted, or -1 (nothing done) when more than
 * cap would be. */
int64_t orc_evict(orc_volume *v, const int32_t lo[3], const int32_t hi[3], int32_t *keys_out, double *T_out,
                  double *P_out, int64_t cap)
{
    int64_t n_out = 0;
    for (int64_t b = 0; b < v->n_blocks; ++b) {
        int inside = 1;
        for (int a = 0; a < 3; ++a) inside &= v->keys[3 * b + a] >= lo[a] && v->keys[3 * b + a] <= hi[a];
        n_out += !inside;
    }
    if (n_out > cap) return -1;
    int64_t kept = 0, e = 0;
    for (int64_t b = 0; b < v->n_blocks; ++b) {
        int inside = 1;
        for (int a = 0; a < 3; ++a) inside &= v->keys[3 * b + a] >= lo[a] && v->keys[3 * b + a] <= hi[a];
        v->offset[table_index(v, v->keys[3 * b], v->keys[3 * b + 1], v->keys[3 * b + 2])] = -1;
        if (!inside) {
            memcpy(keys_out + 3 * e, v->keys + 3 * b, sizeof(int32_t) * 3);
            memcpy(T_out + BVOX * e, v->T + BVOX * b, sizeof(double) * BVOX);
            memcpy(P_out + BVOX * e, v->P + BVOX * b, sizeof(double) * BVOX);
            ++e;
            continue;
        }
        if (kept != b) {
            memcpy(v->keys + 3 * kept, v->keys + 3 * b, sizeof(int32_t) * 3);
            memmove(v->T + BVOX * kept, v->T + BVOX * b, sizeof(double) * BVOX);
            memmove(v->P + BVOX * kept, v->P + BVOX * b, sizeof(double) * BVOX);
        }
        ++kept;
    }
    v->n_blocks = kept;
    for (int64_t b = 0; b < kept; ++b)
        v->offset[table_index(v, v->keys[3 * b], v->keys[3 * b + 1], v->keys[3 * b + 2])] = (int32_t)b;
    return e;
}

int orc_set_block(orc_volume *v, const int32_t key[3], const double *T, const double *P)
{
    for (int a = 0; a < 3; ++a)
        if (key[a] < 0 || key[a] >= v->N[a]) return ORC_EINVAL;
    int64_t b = block_of(v, key[0], key[1], key[2], 1, NULL);
    if (b < 0) return ORC_EFULL;
    for (int k = 0; k < BVOX; ++k) {
        v->T[b * BVOX + k] = T[k];
        v->P[b * BVOX + k] = P ? P[k] : 0.0;
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------- accessors */

void orc_geometry(const orc_volume *v, int32_t dims[3], double *voxel_size, double origin[3])
{
    for (int a = 0; a < 3; ++a) {
        dims[a] = v->G[a];
        origin[a] = v->origin[a];
    }
    *voxel_size = v->vs;
}

int orc_block_key(const orc_volume *v, int64_t b, int32_t key[3])
{
    if (b < 0 || b >= v->n_blocks) return ORC_EINVAL;
    for (int a = 0; a < 3; ++a) key[a] = v->keys[3 * b + a];
    return ORC_OK;
}

int orc_voxel(const orc_volume *v, int32_t gx, int32_t gy, int32_t gz, double *T)
{
    if (gx < 0 || gy < 0 || gz < 0 || gx >= v->G[0] || gy >= v->G[1] || gz >= v->G[2]) return 0;
    int32_t b = v->offset[table_index(v, gx / BLOCK, gy / BLOCK, gz / BLOCK)];
    if (b < 0) return 0;
    *T = v->T[(int64_t)b * BVOX + (gx % BLOCK) + BLOCK * (gy % BLOCK) + BLOCK * BLOCK * (gz % BLOCK)];
    return 1;
}

/*
 * CPU oracle for sparse TSDF fusion and raycasting — TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision restatement of what the method computes:
 * the truncated signed distance of Eq. (1), the block-sparse storage with a
 * dense per-block offset table (Section 4, Fig. 4-5), the projective
 * measurement of Section 7.1, the Kalman update of Algorithm 3, the
 * allocation rule of the Fig. 4 caption and the raycast of Section 5.
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no code with the HIP library.
 *
 * Units: distances are stored normalised by the truncation distance delta
 * (T_hat = T / delta) and variances by delta^2 (P_hat = P / delta^2).  The
 * sentinel chi is the value 2.0; any |T_hat| > 1 means chi.
 */
#ifndef TSDF_ORACLE_H
#define TSDF_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_volume orc_volume;

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_EFULL = 3 };
enum { ORC_NOISE_QUADRATIC = 0, ORC_NOISE_CONSTANT = 1, ORC_NOISE_PER_PIXEL = 2 };
enum { ORC_HIT = 1, ORC_AMBIGUOUS = 2, ORC_BISECT_INVALID = 4, ORC_MARGINAL = 8 };

typedef struct {
    int64_t updates;        /* Algorithm 3 executions (voxels with T_k != chi) */
    int64_t new_blocks;     /* blocks allocated by this frame */
    int64_t ties;           /* decisions with an FP64 margin below 1e-9 */
    int64_t visited;        /* voxels whose measurement was evaluated */
} orc_stats;

orc_volume *orc_create(const int32_t dims[3], double voxel_size, const double origin[3],
                       double trunc_voxels, double q_hat, int64_t capacity_blocks);
void orc_destroy(orc_volume *v);
int64_t orc_block_count(const orc_volume *v);

/* One frame: measurement, allocation and Algorithm 3 for every voxel whose
 * projective measurement is not chi.  depth is [H][W] metres (<= 0 or
 * non-finite = no measurement); K = {fx, fy, cx, cy}; pose is camera-to-world
 * row-major 3x4.  noise_kind selects the measurement variance:
 *   QUADRATIC: sigma = coeff * D^2, p = sigma^2
 *   CONSTANT : p_hat = coeff (already in delta^2 units)
 *   PER_PIXEL: p_hat = phat_px[j*W+i] (delta^2 units)
 * Returns ORC_EFULL (and stops) when the block store is exhausted. */
/* Threads of later integrations (default 1, the serial loop over pixels).
 * More threads split the rows of pixels; the results are the same, only
 * the allocation order of new blocks may differ. */
int orc_set_threads(orc_volume *v, int32_t n_threads);
int orc_integrate(orc_volume *v, const float *depth, int32_t W, int32_t H, const double K[4],
                  const double pose[12], int32_t noise_kind, double coeff, const double *phat_px,
                  orc_stats *st);

/* Raycast selected pixels (pixels = n pairs (i, j); NULL = all W*H in row
 * order).  vertex/normal: n*4 doubles, world frame, w = 1 on a hit, all 0 on
 * a miss.  flags: ORC_* bits per pixel.  n_threads > 1 splits pixels over
 * OpenMP threads (results do not depend on it). */
int orc_raycast(const orc_volume *v, int32_t W, int32_t H, const double K[4], const double pose[12],
                const int32_t *pixels, int64_t n, double *vertex, double *normal, int32_t *flags,
                int32_t n_threads);

/* Interpolated distance F at a world point; returns 0 when F is invalid. */
int orc_sample(const orc_volume *v, const double p[3], double *F);

/* Block store access, in allocation order: keys n*3 (block coordinates),
 * T and P n*512 in voxel order x + 8y + 64z. */
int64_t orc_export(const orc_volume *v, int32_t *keys, double *T, double *P, int64_t cap);
/* Remove every block outside the block-coordinate box [lo, hi] (inclusive),
 * copying it out first (keys_out n*3, T_out and P_out n*512, allocation
 * order); the others keep their order.  Returns n, or -1 if n > cap. */
int64_t orc_evict(orc_volume *v, const int32_t lo[3], const int32_t hi[3], int32_t *keys_out, double *T_out,
                  double *P_out, int64_t cap);
/* Allocate (if needed) block (bx, by, bz) and overwrite its 512 voxels. */
int orc_set_block(orc_volume *v, const int32_t key[3], const double *T, const double *P);

/* Learned noise model (mlp.c): 4-32-32-1 SiLU perceptron predicting
 * log sigma^2 (m^2) from per-pixel features; bf16 rounding at fixed points. */
int orc_mlp_param_count(void);
double orc_bf16(double x);
void orc_mlp_features(const float *depth, int32_t W, int32_t H, const double K[4], double *feat, int32_t *valid);
void orc_mlp_forward(const double *params, const double *x, int64_t n, double *s);
double orc_mlp_loss_grad(const double *params, const double *x, const double *r, int64_t n, double *grad,
                         int32_t round_bf16);

/* Update algorithm of later integrations.  KALMAN: Algorithm 3 (state T,
 * variance P).  RUNNING: Algorithm 1, T <- (1 - w) T + w T_k with constant
 * w in (0, 1]; P is not used.  WEIGHTED: Algorithm 2 with w_k = w (CONSTANT)
 * or w_k = 1 / p_k (INV_VARIANCE, the measurement variance in delta^2 units)
 * and the weight sum W, capped at w_max, stored in P's place. */
enum { ORC_RULE_KALMAN = 0, ORC_RULE_RUNNING = 1, ORC_RULE_WEIGHTED = 2 };
enum { ORC_WEIGHT_CONSTANT = 0, ORC_WEIGHT_INV_VARIANCE = 1 };
int orc_set_rule(orc_volume *v, int32_t rule, int32_t weight_kind, double w, double w_max);

/* Scalar update rules (normalised units, chi = any |T| > 1). */
void orc_alg1_step(double *T, double Tk, double w);
void orc_alg2_step(double *T, double *Wsum, double Tk, double w, double w_max);
void orc_alg3_step(double *T, double *P, double Tk, double pk, double q);

/* Grid of the volume: voxels per axis, voxel edge (m), min corner (m). */
void orc_geometry(const orc_volume *v, int32_t dims[3], double *voxel_size, double origin[3]);
/* Coordinates of the b-th block in allocation order. */
int orc_block_key(const orc_volume *v, int64_t b, int32_t key[3]);
/* Stored T_hat of voxel g: returns 1 when its block is allocated, else 0. */
int orc_voxel(const orc_volume *v, int32_t gx, int32_t gy, int32_t gz, double *T);

/* Marching cubes over the allocated blocks (mc.c).  The case table: for
 * cube index c (bit k set when corner k is inside, F < 0; corner k at offset
 * (k & 1, k >> 1 & 1, k >> 2 & 1)), up to ORC_MC_MAX_TRIS triangles given by
 * cube-edge numbers, -1 terminated; edge 4a + m runs along axis a from the
 * corner whose other two coordinates are (m & 1, m >> 1) in increasing axis
 * order.  Returns the number of triangles of case c. */
#define ORC_MC_MAX_TRIS 8
int orc_mc_case(int32_t c, int32_t edges[3 * ORC_MC_MAX_TRIS]);
/* Triangles of every cell of the grid whose eight corners are valid (block
 * allocated, |T_hat| <= 1).  Cells are visited block by block in allocation
 * order, cells of a block in order x + 8y + 64z (cell g spans voxel centres
 * g .. g + 1).  Per triangle: vid[3] vertex ids 3 * (gx + G0 (gy + G1 gz)) + a
 * of the crossed edge (from voxel g along axis a), t[3] the edge parameter
 * F(g) / (F(g) - F(g + e_a)), pos[9] world positions.  Writes min(n, cap)
 * triangles (any output may be NULL) and returns n. */
int64_t orc_marching_cubes(const orc_volume *v, int64_t *vid, double *t, double *pos, int64_t cap);

#ifdef __cplusplus
}
#endif
#endif

/*
 * libtsdf — point-to-plane ICP on raycast maps (gfx950).
 *
 * Section 6: the live depth map is registered to the scene model rendered by
 * the raycast (vertex and normal maps) with the Chen-Medioni point-to-plane
 * functional, projective matching, and rejection by distance and by normal
 * deviation.  One call is one iteration:
 *
 *   1. every live pixel with a valid depth and valid right and lower
 *      neighbours gives a point p (back-projected through its centre) and a
 *      normal (lower difference x right difference), moved to the world frame
 *      by the current pose estimate;
 *   2. p is projected into the camera the model maps were rendered from and
 *      takes the model vertex q and normal n of the nearest pixel (rounding
 *      floor(u + 1/2), as in fusion);
 *   3. the pair is kept when the model pixel holds a surface, |p - q| <=
 *      dist_max and the live and model normals are at most acos(cos_min)
 *      apart (both tested in double precision without contractions);
 *   4. the pairs' 6x6 normal equations of sum ((R p + t - q) . n)^2 with
 *      c = p x n, the small-angle rotation (alpha, beta, gamma) and t;
 *   5. with shrink set, the system of the unit-cube-scaled problem: m and S
 *      are the centre and extents of the box around every kept p and q, and
 *      c^ = S^-1 (c - m x n);
 *   6. eigen-thresholding: only eigen-directions whose eigenvalue divided by
 *      the number of pairs exceeds theta (0.005 in the paper) contribute to
 *      the solution, sum v (v . b) / lambda;
 *   7. back-substitution r = S^-1 r^, t = t^ - r x m (the inverse of the
 *      substitution in step 5; the relations printed next to the scaled
 *      system do not invert it), then the pose becomes
 *      R' = Rz(gamma) Ry(beta) Rx(alpha) R and t' = Rz Ry Rx t + t_inc.
 *      With no pair the pose is copied unchanged.
 *
 * Steps 1-4 run in one pass over the pixels that writes per-workgroup partial
 * sums.  The pass accumulates the unscaled sums and the box; the scaled
 * system is obtained from them exactly, by the same linear change of
 * variables, in a second single-workgroup kernel that also solves, so the
 * maps are read once.  The paper reads the reduced system back and solves on
 * the CPU; here the 6x6 eigen-decomposition (cyclic Jacobi, double
 * precision) runs on the device and nothing is synchronised.  Successive
 * iterations chain by passing a result's pose as the next call's pose, or
 * all at once through tsdf_icp_run.
 *
 * Conventions are those of tsdf.h.
 */
#ifndef TSDF_ICP_H
#define TSDF_ICP_H

#include "tsdf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double dist_max;   /* metres, > 0 */
    double cos_min;    /* in [-1, 1] */
    double theta;      /* eigenvalue threshold per pair; < 0 keeps every direction with a positive eigenvalue */
    int32_t shrink;    /* 1: solve the unit-cube-scaled system, 0: the system as it stands */
    int32_t pad;
} tsdf_icp_params;

/* Written by the device at the end of each iteration. */
typedef struct {
    double pose[12];     /* updated camera-to-world pose, row-major 3x4 */
    double x[6];         /* increment applied: alpha, beta, gamma (rad), t (m) */
    double lambda[6];    /* eigenvalues of the solved system divided by the pair count, ascending */
    double C[36];        /* the solved system matrix (scaled when shrink is set), row-major */
    double b[6];         /* its right-hand side */
    double m[3];         /* box centre (zero without shrink) */
    double S[3];         /* box extents, 1 where an extent is 0 (ones without shrink) */
    double residual2;    /* sum over pairs of ((p - q) . n)^2 before the update */
    int64_t pairs;       /* number of kept pairs */
    int32_t kept;        /* number of eigen-directions kept */
    int32_t pad;
} tsdf_icp_result;

/* Device workspace that tsdf_icp_step and tsdf_icp_run need for a width x
 * height depth map (0 if a dimension is outside 1..16384): per-workgroup
 * partial sums and the last iteration's eigenvectors. */
uint64_t tsdf_icp_workspace_bytes(int32_t width, int32_t height);

/* One iteration.
 *   depth_dev         float32 [H][W] live depth map (device)
 *   K                 intrinsics of both the live map and the model maps (host)
 *   model_vertex_dev  float4 [H][W] world vertices, w = 1 where valid (device),
 *   model_normal_dev  float4 [H][W] unit world normals (device): tsdf_raycast output
 *   model_pose_c2w    pose the model maps were rendered from (host, 12 doubles)
 *   pose_dev          current estimate of the live pose (device, 12 doubles);
 *                     it may be result_dev->pose
 *   params            host
 *   workspace_dev     at least tsdf_icp_workspace_bytes(W, H) bytes (device)
 *   result_dev        device
 * Returns TSDF_EINVAL for null pointers, invalid intrinsics or model pose,
 * non-finite or out-of-range parameters, or a small workspace; nothing is
 * enqueued then. */
tsdf_status tsdf_icp_step(const float *depth_dev, const tsdf_intrinsics *K, const float *model_vertex_dev,
                          const float *model_normal_dev, const double model_pose_c2w[12], const double *pose_dev,
                          const tsdf_icp_params *params, void *workspace_dev, uint64_t workspace_bytes,
                          tsdf_icp_result *result_dev, hipStream_t stream);

/* `iters` chained iterations (1..1024) from the host pose pose_init_c2w (12
 * doubles, read during the call): iteration 0 starts from it, iteration k
 * from results_dev[k - 1].pose.  results_dev holds `iters` records (device).
 * Enqueues 2 * iters kernels and no copy.  Iterations after the first start
 * their eigen-decomposition from the previous iteration's eigenvectors (kept
 * in the workspace), which the nearly unchanged system needs only a sweep or
 * two to finish; the result is the same decomposition to rounding.  Same
 * errors as tsdf_icp_step, and TSDF_EINVAL for an initial pose that is not a
 * finite rotation (as the model pose) or iters out of range. */
tsdf_status tsdf_icp_run(const float *depth_dev, const tsdf_intrinsics *K, const float *model_vertex_dev,
                         const float *model_normal_dev, const double model_pose_c2w[12],
                         const double pose_init_c2w[12], const tsdf_icp_params *params, int32_t iters,
                         void *workspace_dev, uint64_t workspace_bytes, tsdf_icp_result *results_dev,
                         hipStream_t stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * allocation-free serving loops): tsdf_icp_run without a workspace argument.
 * Its partial sums and warm-start eigenvectors live in a static array of the
 * library, 164,128 bytes per device (the partials of at most 512 workgroups,
 * enough for every frame size tsdf_icp_workspace_bytes accepts), reserved on
 * each device the library runs on until the process ends.  The call
 * allocates nothing.  Results are bitwise those of tsdf_icp_run with a
 * workspace.  All calls on one device share that array, so calls whose work
 * may overlap on one device (several streams, or several host threads) race
 * and must be serialised by the caller.  Same arguments and errors as
 * tsdf_icp_run; TSDF_EINVAL also for a frame size outside 1..16384 per axis,
 * TSDF_EHIP when the array's device address cannot be obtained. */
tsdf_status tsdf_icp_run_noalloc(const float *depth_dev, const tsdf_intrinsics *K, const float *model_vertex_dev,
                                 const float *model_normal_dev, const double model_pose_c2w[12],
                                 const double pose_init_c2w[12], const tsdf_icp_params *params, int32_t iters,
                                 tsdf_icp_result *results_dev, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif

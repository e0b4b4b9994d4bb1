/*
 * libtsdf — batched multi-scene step (gfx950).
 *
 * Many independent reconstructions advance together: one step fuses one
 * depth map into each scene's volume (Section 7.1 with Algorithm 3, block
 * allocation of Section 7.2) and raycasts each volume from the same pose
 * (Section 5), exactly as tsdf_integrate_frame followed by tsdf_raycast would,
 * but with six kernel launches that cover every scene instead of five per
 * scene, or with one cooperative launch (tsdf_batch_set_persistent).  The
 * paper handles one sensor stream; batching is an addition for serving many
 * small scenes at once, where per-scene launches would leave most of the chip
 * idle.  Results per scene are bitwise identical to the single-volume calls.
 *
 * The step can be captured into a hipGraph once and replayed; per-step inputs
 * travel in a small device table (tsdf_batch_bytes, caller-owned) that each
 * step rewrites before it launches.
 *
 * Conventions are those of tsdf.h.  A batch holds 1..64 volumes, all with the
 * same storage type and index mode, each volume at most once; it does not own
 * them.  Each scene keeps its own intrinsics, fixed at creation (width and
 * height within the volume's maxima).  While a batch is in use its volumes are
 * driven only through it, from one stream.
 */
#ifndef TSDF_BATCH_H
#define TSDF_BATCH_H

#include "tsdf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tsdf_batch tsdf_batch;

/* Device bytes of the per-step table for n_scenes scenes (0 if n_scenes is
 * outside 1..64). */
uint64_t tsdf_batch_bytes(int32_t n_scenes);

/* Create a batch over vols[0..n) with intrinsics K[0..n) (host arrays, read
 * during the call).  dev_buf: device memory of at least tsdf_batch_bytes(n)
 * bytes, owned by the caller, alive as long as the batch.  Returns
 * TSDF_EINVAL for null or repeated volumes, invalid or oversized intrinsics,
 * mixed storage types or index modes, or a small buffer.  Graph capture is
 * off and the raycast group is 8 after creation. */
tsdf_status tsdf_batch_create(tsdf_volume *const *vols, const tsdf_intrinsics *K, int32_t n, void *dev_buf,
                              uint64_t bytes, tsdf_batch **out);
void tsdf_batch_destroy(tsdf_batch *b);

/* Capture the step into a hipGraph on first use and replay it afterwards
 * (re-captured when the noise kind or raycast group changes).  Graph mode
 * needs a created (non-null) stream. */
tsdf_status tsdf_batch_set_graph(tsdf_batch *b, int32_t enable);

/* Persistent mode (enable != 0): the whole step runs as one cooperative
 * launch of a resident grid (as many 256-thread workgroups as can be
 * resident at once), its six phases separated by grid barriers; each phase
 * uses the same kernel bodies and work decomposition as the six launches, so
 * results are bitwise those of the default mode.  Graph capture does not
 * apply to this mode (the step is one launch already).  TSDF_EINVAL for a
 * batch of volumes without the dense block index.  A step returns TSDF_EHIP
 * if the device cannot run the cooperative launch. */
tsdf_status tsdf_batch_set_persistent(tsdf_batch *b, int32_t enable);

/* Lanes per ray of the batched raycast (1, 2, 4, 8 or 16). */
tsdf_status tsdf_batch_set_raycast_group(tsdf_batch *b, int32_t group);
int32_t tsdf_batch_get_raycast_group(const tsdf_batch *b);

/* One step.  Host arrays of n entries: depth_dev[k] the scene's depth map
 * (float32 [H_k][W_k], device) or null to leave scene k untouched this step;
 * poses_c2w 12 n doubles, scene k's pose at 12 k (used both to fuse and to
 * raycast); vertex_dev[k], normal_dev[k] float4 [H_k][W_k] outputs (device).
 * noise applies to every scene (null means quadratic with coeff 0).  Fails
 * with TSDF_EFULL, enqueuing nothing, when a volume has a sticky flag that
 * tsdf_query_stats has seen.  Argument errors enqueue nothing. */
tsdf_status tsdf_batch_step(tsdf_batch *b, const float *const *depth_dev, const double *poses_c2w,
                            float *const *vertex_dev, float *const *normal_dev, const tsdf_noise_model *noise,
                            hipStream_t stream);

/* Autotuner of the batched raycast: raycasts every scene from poses_c2w with
 * each group size (reps timed repetitions after one warm-up), keeps the
 * fastest and reports it with the mean time of one batched raycast in
 * milliseconds.  Synchronises `stream`; the outputs hold the last raycast. */
tsdf_status tsdf_batch_autotune_raycast(tsdf_batch *b, const double *poses_c2w, float *const *vertex_dev,
                                        float *const *normal_dev, int32_t reps, hipStream_t stream,
                                        int32_t *best_group, float *best_ms);

/* Workgroups of the batched fusion launch (1..65536; 2560 after creation):
 * the fusion walks every scene's candidate blocks with this many persistent
 * workgroups of four wavefronts.  Results do not depend on it. */
tsdf_status tsdf_batch_set_fuse_grid(tsdf_batch *b, uint32_t workgroups);
uint32_t tsdf_batch_get_fuse_grid(const tsdf_batch *b);

/* Autotuner of the fusion grid: runs whole steps (six launches, one warm-up
 * and `reps` timed per candidate) on the given frames with each candidate
 * grid, keeps the fastest and reports it with the mean time of one step in
 * milliseconds.  The frames are fused 5 (1 + reps) times into the volumes
 * (five candidates): tune on warm-up data and reset the volumes afterwards.  Arguments as
 * tsdf_batch_step; synchronises `stream`. */
tsdf_status tsdf_batch_autotune_fuse(tsdf_batch *b, const float *const *depth_dev, const double *poses_c2w,
                                     float *const *vertex_dev, float *const *normal_dev,
                                     const tsdf_noise_model *noise, int32_t reps, hipStream_t stream,
                                     uint32_t *best_grid, float *best_ms);

#ifdef __cplusplus
}
#endif
#endif

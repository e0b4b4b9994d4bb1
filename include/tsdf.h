/*
 * libtsdf — block-sparse TSDF fusion and raycasting on AMD Instinct MI355X (gfx950).
 *
 * The method is that of "Real-time High Resolution Fusion of Depth Maps on
 * GPU" (Trifonov, arXiv:1311.7194):
 *   - Eq. (1): a truncated signed distance, positive outside the surface,
 *     replaced by the sentinel chi beyond the truncation distance delta;
 *   - Section 4 and Fig. 4: the field is split into blocks of 8^3 voxels and
 *     only blocks that store something other than chi take memory;
 *   - Section 7.1: each frame contributes the projective measurement T_k(x)
 *     (project x into the depth map, take the distance to the sample there)
 *     and Algorithm 3 fuses it with a per-voxel Kalman filter (state T,
 *     variance P, measurement variance p_k, process variance Q);
 *   - Section 7.2: blocks intersected by the measured surface are allocated,
 *     other blocks in view are updated only if already allocated;
 *   - Section 5: raycasting the sparse field yields vertex and normal maps.
 *
 * Conventions shared by every entry point
 *   Pose: camera-to-world, row-major 3x4 [R | t] in double precision
 *     (x_world = R x_cam + t).  Camera axes x right, y down, z forward.
 *   Pixels: (i, j) = (column, row), centre at image point (i, j); a voxel
 *     projects to the pixel with the nearest centre.
 *   Depth: float32 [height][width], metres along camera z; <= 0, NaN or Inf
 *     means no measurement.
 *   Grid: voxel g in [0, dims) has its centre at origin + (g + 0.5) * voxel_size.
 *   Stored values are normalised: T_hat = T / delta in [-1, 1] and
 *     P_hat = P / delta^2; chi is stored as T_hat = 2.
 *   Device pointers ("_dev") are HIP device memory owned by the caller; the
 *     library never allocates device memory.  Host pointers are read during
 *     the call only.
 *   Streams: every call that takes a hipStream_t enqueues its work on that
 *     stream and returns without synchronising; buffers passed in must stay
 *     valid until the work completes.  One volume is driven from one stream
 *     at a time.
 *   Errors: argument errors return synchronously and enqueue nothing.
 *     Exhaustion detected on the device (block pool, hash table, per-frame
 *     candidate list) latches a sticky device flag.  The library does not
 *     synchronise to look at it: tsdf_query_stats reads it, and once it has
 *     seen a flag, tsdf_integrate_frame returns TSDF_EFULL until
 *     tsdf_reset_volume.  No C++ exception crosses this interface.
 */
#ifndef TSDF_H
#define TSDF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TSDF_OK = 0,
    TSDF_EINVAL = 1,   /* bad argument (null, size, non-finite or non-orthonormal pose, ...) */
    TSDF_ENOMEM = 2,   /* caller buffer smaller than tsdf_volume_bytes reports */
    TSDF_EFULL = 3,    /* pool, hash or candidate list exhausted (sticky) */
    TSDF_EHIP = 4,     /* a HIP runtime call failed */
    TSDF_ESTATE = 5    /* call not valid in the current state */
} tsdf_status;

typedef enum { TSDF_F32 = 0, TSDF_F16 = 1 } tsdf_storage;

/* Sticky device status bits (tsdf_stats.status_flags). */
enum { TSDF_FLAG_POOL_FULL = 1u, TSDF_FLAG_HASH_FULL = 2u, TSDF_FLAG_CAND_FULL = 4u };

typedef struct {
    int32_t dims[3];           /* virtual grid in voxels, each a positive multiple of 8, <= 8192 */
    double voxel_size;         /* metres */
    double origin[3];          /* world position of the grid's min corner, metres */
    double trunc_voxels;       /* delta = trunc_voxels * voxel_size */
    uint32_t capacity_blocks;  /* block pool size, 1 .. 2^22 */
    uint32_t hash_slots;       /* power of two >= 2 * capacity_blocks */
    int32_t storage;           /* tsdf_storage: T_hat and P_hat as float32 or float16 */
    double q_hat;              /* process variance Q / delta^2 (Algorithm 3) */
    int32_t max_width;         /* largest frame the volume will see */
    int32_t max_height;
    uint32_t max_candidates;   /* candidate blocks per frame; 0 = capacity_blocks */
    int32_t dense_index;       /* 1: also keep a dense per-block index (4 bytes per virtual block,
                                  the offset buffer of Section 4) for single-load lookups in the
                                  raycast; 0: look blocks up through the hash only */
} tsdf_volume_desc;

typedef struct {
    double fx, fy, cx, cy;     /* pixels */
    int32_t width, height;
} tsdf_intrinsics;

typedef enum {
    TSDF_NOISE_QUADRATIC = 0,  /* sigma = coeff * D^2, p = sigma^2 (Section 7.1) */
    TSDF_NOISE_CONSTANT = 1,   /* p_hat = coeff, already in delta^2 units */
    TSDF_NOISE_MLP = 2         /* learned per-pixel variance, quadratic fallback (tsdf_mlp.h) */
} tsdf_noise_kind;

/* Update algorithm that fuses measurements (tsdf_set_update_rule). */
typedef enum {
    TSDF_RULE_KALMAN = 0,      /* Algorithm 3: state T, variance P (default) */
    TSDF_RULE_RUNNING = 1,     /* Algorithm 1: T <- (1 - w) T + w T_k, constant w in (0, 1]; P unused (0) */
    TSDF_RULE_WEIGHTED = 2     /* Algorithm 2: weighted mean, weight sum W capped at w_max, stored in P */
} tsdf_update_rule;

typedef enum {
    TSDF_WEIGHT_CONSTANT = 0,      /* w_k = w */
    TSDF_WEIGHT_INV_VARIANCE = 1   /* w_k = 1 / p_hat_k, the measurement variance of the noise model */
} tsdf_weight_kind;

typedef struct {
    int32_t kind;              /* tsdf_noise_kind */
    double coeff;              /* see tsdf_noise_kind; the MLP uses it for its fallback */
    const void *mlp_params_dev;/* TSDF_NOISE_MLP: packed parameters, see tsdf_mlp.h */
} tsdf_noise_model;

typedef struct {
    uint64_t allocated_blocks;    /* blocks in the pool */
    uint64_t frame_candidates;    /* candidate blocks examined by the last integrate */
    uint64_t frame_new_blocks;    /* blocks allocated by the last integrate */
    uint64_t frame_updates;       /* voxel updates (update-rule executions) in the last integrate */
    uint64_t frame_fresh_updates; /* ... of which in blocks that frame allocated */
    uint64_t total_updates;       /* totals since creation or reset */
    uint64_t total_fresh_updates;
    uint64_t total_candidates;
    uint64_t total_new_blocks;
    uint64_t frames;              /* integrate calls since creation or reset */
    uint64_t frame_touched_blocks;/* blocks that received an update in the last integrate */
    uint64_t total_touched_blocks;
    uint32_t status_flags;        /* TSDF_FLAG_* (sticky) */
    uint32_t reserved;
} tsdf_stats;

/* Per-stage kernel times from HIP events recorded around each launch while
 * timing is enabled: pixel preparation, block fusion, the raycast's range
 * pass (span reset and per-block projection) and the raycast march itself. */
typedef struct {
    double prep_ms, fuse_ms, range_ms, raycast_ms;
    uint64_t prep_launches, fuse_launches, range_launches, raycast_launches;
} tsdf_timing;

typedef struct tsdf_volume tsdf_volume;

/* Device bytes a volume needs (pool, hash table, occupancy bitmaps, per-frame
 * scratch).  Returns TSDF_EINVAL for an invalid description. */
tsdf_status tsdf_volume_bytes(const tsdf_volume_desc *desc, uint64_t *bytes);

/* Create a volume in the caller's device buffer dev_buf (>= tsdf_volume_bytes,
 * 256-byte aligned).  Clears the buffer on `stream`.  The host handle is
 * written to *out and released by tsdf_destroy_volume. */
tsdf_status tsdf_create_volume(const tsdf_volume_desc *desc, void *dev_buf, uint64_t bytes,
                               hipStream_t stream, tsdf_volume **out);
void tsdf_destroy_volume(tsdf_volume *vol);

/* Empty the volume (all blocks released, counters and sticky flags cleared). */
tsdf_status tsdf_reset_volume(tsdf_volume *vol, hipStream_t stream);

/* Fuse one depth map (Section 7): allocate every block holding a voxel whose
 * measurement is not chi (Fig. 4 caption), then apply Algorithm 3 to every
 * such voxel.  depth_dev: float32 [K->height][K->width] (width <= max_width,
 * height <= max_height).  pose_c2w: host, 12 doubles.  noise: host. */
tsdf_status tsdf_integrate_frame(tsdf_volume *vol, const float *depth_dev, const tsdf_intrinsics *K,
                                 const double pose_c2w[12], const tsdf_noise_model *noise,
                                 hipStream_t stream);

/* Raycast the volume (Section 5) from pose_c2w into float4 maps
 * [K->height][K->width][4] (any frame size): vertex (x, y, z, 1) and unit
 * normal (x, y, z, 1) in world coordinates; both all zero where the ray finds
 * no front-facing zero crossing or the normal is undefined.  The ray through
 * each pixel centre is sampled every half voxel from the camera centre; the
 * first bracket with F > 0 >= F over valid trilinear samples is refined by
 * six quaternary search steps and a final linear interpolation; the normal is the central difference of F one voxel apart
 * along the world axes. */
tsdf_status tsdf_raycast(tsdf_volume *vol, const tsdf_intrinsics *K, const double pose_c2w[12],
                         float *vertex_dev, float *normal_dev, hipStream_t stream);

/* The raycast above, also counting the blocks whose voxels the rays' march
 * samples are based in (each block once, however many rays read it).  This
 * is the data the raycast must read from the pool: the measure of its
 * algorithmic traffic.  The maps are bitwise those of tsdf_raycast.  Runs an
 * instrumented copy of the march (not the one tsdf_raycast times) and
 * synchronises `stream` to return *blocks_out. */
tsdf_status tsdf_raycast_footprint(tsdf_volume *vol, const tsdf_intrinsics *K, const double pose_c2w[12],
                                   float *vertex_dev, float *normal_dev, uint64_t *blocks_out,
                                   hipStream_t stream);

/* Update algorithm of later integrations (Section 7.1): Algorithm 3 (the
 * default), Algorithm 1 with constant weight w in (0, 1] (weight_kind must be
 * TSDF_WEIGHT_CONSTANT), or Algorithm 2 with w_k = w > 0 or w_k = 1 / p_hat_k
 * and the weight sum capped at w_max > 0 (may be +Inf with FP32 storage; at
 * most 65504 with FP16 storage, where stored weights are clamped to 65504).
 * Allocation does not depend on the rule.  P holds the Kalman variance, 0
 * (Algorithm 1) or the weight sum W (Algorithm 2): switching rules on a
 * volume that holds data reinterprets it, so set the rule after creation or
 * tsdf_reset_volume (which keeps it).  With inverse-variance weights and no
 * cap, Algorithm 2 is Algorithm 3 with Q = 0 (P = 1/W).  Host-side: takes
 * effect for calls enqueued afterwards.  TSDF_EINVAL for other values. */
tsdf_status tsdf_set_update_rule(tsdf_volume *vol, int32_t rule, int32_t weight_kind, double w, double w_max);

/* Lanes that march one ray together in the raycast (1, 2, 4, 8 or 16; default 8).
 * Every group size gives bitwise the same maps; only the speed differs. */
tsdf_status tsdf_set_raycast_group(tsdf_volume *vol, int32_t group);
int32_t tsdf_get_raycast_group(const tsdf_volume *vol);

/* Autotuner: raycasts the current volume from pose_c2w with every group size
 * (`reps` timed launches each after one warm-up, HIP events on `stream`),
 * keeps the fastest for later raycasts and reports it with its mean time in
 * milliseconds.  Synchronises `stream`.  The outputs hold the last raycast. */
tsdf_status tsdf_autotune_raycast(tsdf_volume *vol, const tsdf_intrinsics *K, const double pose_c2w[12],
                                  float *vertex_dev, float *normal_dev, int32_t reps, hipStream_t stream,
                                  int32_t *best_group, float *best_ms);

/* Counters and sticky flags; synchronises the stream the volume last used. */
tsdf_status tsdf_query_stats(tsdf_volume *vol, tsdf_stats *out);

/* Enable (1) or disable (0) per-launch event timing.  While enabled every
 * kernel launch is bracketed by two HIP events on its stream. */
tsdf_status tsdf_set_timing(tsdf_volume *vol, int32_t enable);
/* Sum of the recorded kernel times (synchronises on the events); reset != 0
 * clears the sums. */
tsdf_status tsdf_read_timing(tsdf_volume *vol, tsdf_timing *out, int32_t reset);

/* Copy out the allocated blocks in pool order: keys_dev int32 [cap][3]
 * (block coordinates), T_dev and P_dev [cap][512] of the storage type, voxel
 * order x + 8y + 64z.  *n_out (host) receives the block count; the call
 * synchronises `stream` to read it.  Copies min(n, cap) blocks. */
tsdf_status tsdf_export_blocks(tsdf_volume *vol, int32_t *keys_dev, void *T_dev, void *P_dev,
                               uint64_t cap, uint64_t *n_out, hipStream_t stream);

/* Device workspace of tsdf_evict_blocks for this volume (0 for null). */
uint64_t tsdf_evict_workspace_bytes(const tsdf_volume *vol);

/* Block eviction, the volume shift named as future work in Section 8: every
 * allocated block whose block coordinates lie outside [lo, hi] (inclusive,
 * per axis; host arrays) is copied out and removed.  keys_dev int32 [cap][3],
 * T_dev and P_dev [cap][512] of the storage type receive the evicted blocks,
 * in no particular order; *n_out (host) their number.  The kept blocks move
 * to the front of the pool, and the hash table, occupancy bits and dense
 * index are rebuilt from them; their values are unchanged.  A later frame
 * that reaches an evicted block allocates it afresh; tsdf_import_blocks
 * streams evicted blocks back in.  Synchronises `stream` twice.  Returns
 * TSDF_ENOMEM, changing nothing, when more than cap blocks would be evicted
 * (*n_out is then the number needed); TSDF_EFULL as tsdf_integrate_frame. */
tsdf_status tsdf_evict_blocks(tsdf_volume *vol, const int32_t lo[3], const int32_t hi[3], int32_t *keys_dev,
                              void *T_dev, void *P_dev, uint64_t cap, void *work_dev, uint64_t work_bytes,
                              uint64_t *n_out, hipStream_t stream);

/* Insert (or overwrite) n blocks: keys_dev int32 [n][3] distinct block
 * coordinates inside the grid, T_dev/P_dev [n][512] of the storage type. */
tsdf_status tsdf_import_blocks(tsdf_volume *vol, const int32_t *keys_dev, const void *T_dev,
                               const void *P_dev, uint64_t n, hipStream_t stream);

const char *tsdf_status_string(tsdf_status s);

#ifdef __cplusplus
}
#endif
#endif

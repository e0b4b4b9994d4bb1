/*
 * libtsdf — marching-cubes extraction of the fused surface (Section 5 of
 * Trifonov, arXiv:1311.7194: the polygonisation alternative to raycasting,
 * which finds the occupied cells and the number of vertices each produces,
 * turns the counts into output offsets with a prefix sum, and polygonises
 * only the occupied cells).  Conventions as in tsdf.h.
 *
 * Cells and vertices
 *   Cell g spans the voxel centres g + {0,1}^3 (g in [0, dims - 1) per axis)
 *   and is polygonised when all eight corners hold a distance (|T_hat| <= 1)
 *   in allocated blocks.  Corner k sits at offset (k & 1, k >> 1 & 1,
 *   k >> 2 & 1); it is inside when T_hat < 0 (0 counts as outside).  A cell
 *   edge whose corners differ carries one vertex: for the edge from voxel g
 *   along axis a, its id is 3 * (gx + dims[0] * (gy + dims[1] * gz)) + a and
 *   its position is g + 0.5 + t e_a voxels from the grid origin, with
 *   t = T(g) / (T(g) - T(g + e_a)) in [0, 1].  Cells that share an edge share
 *   its vertex id, so ids weld the triangles into a mesh.
 *
 * Case table
 *   Cube edge 4a + m runs along axis a from the corner whose other two
 *   coordinates, in increasing axis order, are (m & 1, m >> 1).  On each cube
 *   face the crossing points are joined in pairs: where the face's inside
 *   corners sit diagonally, each is cut off on its own.  Face segments are
 *   directed with the inside on their right seen from outside the cube, close
 *   into loops, and each loop, started at its smallest edge number, is
 *   fanned from that edge.  Neighbouring cells therefore cut shared faces
 *   alike (no cracks), and triangles wind counter-clockwise seen from the
 *   outside (T_hat > 0).
 */
#ifndef TSDF_MESH_H
#define TSDF_MESH_H

#include "tsdf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* The case table: for cube case c (bit k set when corner k is inside) writes
 * the cube edges of its triangles, three per triangle, -1 after the last, to
 * edges[15] (host) and returns the triangle count (0..5); -1 for c outside
 * 0..255 or a null pointer.  Host only. */
int32_t tsdf_mesh_case(int32_t c, int32_t edges[15]);

/* Device workspace of tsdf_extract_mesh for this volume (0 for null):
 * two counters per pool slot and two per 1024 slots. */
uint64_t tsdf_mesh_workspace_bytes(const tsdf_volume *vol);

/* Triangles of every polygonised cell of the allocated blocks, enqueued on
 * `stream` without synchronising.  count_dev (device, one uint64) receives
 * the number of triangles n; the first min(n, cap) are written:
 *   vertex_id_dev  int64 [cap][3]  vertex ids (see above)
 *   t_dev          float [cap][3]  edge parameters t
 *   xyz_dev        float [cap][3][3] world positions (may be null)
 * Triangles are grouped by block in pool order and, within a block, by cell
 * in x + 8y + 64z order.  A caller that does not know n can call with cap = 0
 * (nothing is written but the count), read it, and call again.  The volume
 * is only read.  TSDF_EINVAL for a null volume or count, a small workspace,
 * or cap > 0 with a null vertex_id_dev or t_dev; TSDF_EFULL as
 * tsdf_integrate_frame. */
tsdf_status tsdf_extract_mesh(tsdf_volume *vol, int64_t *vertex_id_dev, float *t_dev, float *xyz_dev, uint64_t cap,
                              void *work_dev, uint64_t work_bytes, uint64_t *count_dev, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif

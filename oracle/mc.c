/*
 * Marching cubes over the allocated blocks — TEST INFRASTRUCTURE ONLY.
 *
 * Section 5 names marching cubes polygonisation of the non-empty blocks as
 * the alternative to raycasting and splits it into three stages: find the
 * occupied voxels and the number of vertices each produces, turn those
 * counts into output offsets with a prefix sum, then polygonise only the
 * occupied voxels.  This file computes what those stages produce, in one
 * plain pass: every cell, in a fixed order, emits its triangles.
 *
 * The paper names the algorithm (Lorensen and Cline) but prints no case
 * table; the readings taken here:
 *   - a cell spans eight voxel centres g + {0,1}^3; it is valid when all
 *     eight lie in allocated blocks and hold a distance (|T_hat| <= 1);
 *   - a corner is inside when F < 0; F = 0 counts as outside (the usual
 *     marching-cubes convention; the raycast, which stops at the first
 *     F <= 0, puts such a point on its inside, but both place the surface
 *     at the same point);
 *   - a cell edge whose corners differ carries one vertex at the linear
 *     zero of F along it, t = F(lo) / (F(lo) - F(hi)) from its low corner;
 *   - the case table is derived, not transcribed: on each cube face the
 *     crossing points are joined in pairs, and on a face whose inside corners
 *     sit diagonally (the ambiguous face) each inside corner is cut off on
 *     its own; every face segment is directed so that the inside corner it
 *     cuts off lies to its right seen from outside the cube; the segments
 *     close into loops, and each loop, read from its smallest edge number,
 *     is fanned into triangles from that edge.  Neighbouring cells see the
 *     same four values on a shared face, so they cut it the same way and the
 *     surface has no cracks; triangles wind counter-clockwise seen from the
 *     outside (F > 0) side.
 * Plain double precision; the table is built on first use.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

#define NCORNER 8
#define NEDGE 12

/* corner k sits at (k & 1, k >> 1 & 1, k >> 2 & 1) of the unit cube */
static int corner_coord(int k, int a) { return (k >> a) & 1; }

/* the two corners of cube edge e = 4a + m: along axis a, the other two axes
 * (in increasing order) at (m & 1, m >> 1) */
static void edge_corners(int e, int *lo, int *hi)
{
    int a = e / 4, m = e % 4;
    int other[2], n = 0;
    for (int b = 0; b < 3; ++b)
        if (b != a) other[n++] = b;
    int c = ((m & 1) << other[0]) | (((m >> 1) & 1) << other[1]);
    *lo = c;
    *hi = c | (1 << a);
}

static int edge_between(int p, int q)
{
    for (int e = 0; e < NEDGE; ++e) {
        int lo, hi;
        edge_corners(e, &lo, &hi);
        if ((lo == p && hi == q) || (lo == q && hi == p)) return e;
    }
    return -1;
}

static void edge_midpoint(int e, double m[3])
{
    int lo, hi;
    edge_corners(e, &lo, &hi);
    for (int a = 0; a < 3; ++a) m[a] = 0.5 * (corner_coord(lo, a) + corner_coord(hi, a));
}

static int n_tri[256];
static int tri_edges[256][3 * ORC_MC_MAX_TRIS];
static int table_ready;

/* The case table from the rule stated at the top of this file. */
static void build_table(void)
{
    for (int c = 0; c < 256; ++c) {
        int next[NEDGE];
        for (int e = 0; e < NEDGE; ++e) next[e] = -1;
        for (int a = 0; a < 3; ++a) {
            for (int side = 0; side < 2; ++side) {
                /* the face's corners in cyclic order: the two free axes u < v */
                int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
                int base = side << a;
                int q[4] = {base, base | (1 << u), base | (1 << u) | (1 << v), base | (1 << v)};
                int in[4];
                for (int i = 0; i < 4; ++i) in[i] = (c >> q[i]) & 1;
                double n[3] = {0, 0, 0};
                n[a] = side ? 1.0 : -1.0;   /* outward normal of the face */
                int cross = 0;
                for (int i = 0; i < 4; ++i) cross += in[i] != in[(i + 1) % 4];
                if (cross == 0) continue;
                /* each segment: its two edges and the inside corner it cuts off */
                int seg[2][3], nseg = 0;
                if (cross == 2) {
                    int ends[2], k = 0, corner_in = -1;
                    for (int i = 0; i < 4; ++i) {
                        if (in[i] != in[(i + 1) % 4]) ends[k++] = edge_between(q[i], q[(i + 1) % 4]);
                        if (in[i]) corner_in = q[i];
                    }
                    seg[0][0] = ends[0];
                    seg[0][1] = ends[1];
                    seg[0][2] = corner_in;
                    nseg = 1;
                } else { /* four crossings: two diagonal inside corners, each cut off alone */
                    for (int i = 0; i < 4; ++i) {
                        if (!in[i]) continue;
                        seg[nseg][0] = edge_between(q[(i + 3) % 4], q[i]);
                        seg[nseg][1] = edge_between(q[i], q[(i + 1) % 4]);
                        seg[nseg][2] = q[i];
                        ++nseg;
                    }
                }
                for (int s = 0; s < nseg; ++s) {
                    double p0[3], p1[3], m[3], d[3], r[3];
                    edge_midpoint(seg[s][0], p0);
                    edge_midpoint(seg[s][1], p1);
                    for (int k = 0; k < 3; ++k) {
                        d[k] = p1[k] - p0[k];
                        m[k] = 0.5 * (p0[k] + p1[k]);
                        r[k] = corner_coord(seg[s][2], k) - m[k];
                    }
                    /* (d x r) . n < 0: the inside corner lies to the right of d seen from outside */
                    double crs[3] = {d[1] * r[2] - d[2] * r[1], d[2] * r[0] - d[0] * r[2], d[0] * r[1] - d[1] * r[0]};
                    double s_ = crs[0] * n[0] + crs[1] * n[1] + crs[2] * n[2];
                    int from = s_ < 0 ? seg[s][0] : seg[s][1];
                    int to = s_ < 0 ? seg[s][1] : seg[s][0];
                    if (next[from] != -1) abort();   /* each crossing point starts one segment */
                    next[from] = to;
                }
            }
        }
        int used[NEDGE] = {0}, nt = 0;
        for (int e0 = 0; e0 < NEDGE; ++e0) {
            if (next[e0] < 0 || used[e0]) continue;
            int loop[NEDGE], k = 0, e = e0;
            do {
                if (k == NEDGE || used[e] || next[e] < 0) abort();
                used[e] = 1;
                loop[k++] = e;
                e = next[e];
            } while (e != e0);
            for (int i = 1; i + 1 < k; ++i) {
                if (nt == ORC_MC_MAX_TRIS) abort();
                tri_edges[c][3 * nt + 0] = loop[0];
                tri_edges[c][3 * nt + 1] = loop[i];
                tri_edges[c][3 * nt + 2] = loop[i + 1];
                ++nt;
            }
        }
        n_tri[c] = nt;
        for (int i = 3 * nt; i < 3 * ORC_MC_MAX_TRIS; ++i) tri_edges[c][i] = -1;
    }
    table_ready = 1;
}

int orc_mc_case(int32_t c, int32_t edges[3 * ORC_MC_MAX_TRIS])
{
    if (c < 0 || c > 255) return -1;
    if (!table_ready) build_table();
    for (int i = 0; i < 3 * ORC_MC_MAX_TRIS; ++i) edges[i] = tri_edges[c][i];
    return n_tri[c];
}

int64_t orc_marching_cubes(const orc_volume *v, int64_t *vid, double *t, double *pos, int64_t cap)
{
    if (!table_ready) build_table();
    int32_t G[3];
    double vs, origin[3];
    orc_geometry(v, G, &vs, origin);
    int64_t n = 0, nb = orc_block_count(v);
    for (int64_t b = 0; b < nb; ++b) {
        int32_t key[3];
        orc_block_key(v, b, key);
        for (int cz = 0; cz < 8; ++cz)
            for (int cy = 0; cy < 8; ++cy)
                for (int cx = 0; cx < 8; ++cx) {
                    int g[3] = {8 * key[0] + cx, 8 * key[1] + cy, 8 * key[2] + cz};
                    double F[NCORNER];
                    int valid = 1;
                    for (int k = 0; k < NCORNER && valid; ++k) {
                        int ok = orc_voxel(v, g[0] + corner_coord(k, 0), g[1] + corner_coord(k, 1),
                                           g[2] + corner_coord(k, 2), &F[k]);
                        valid = ok && F[k] >= -1.0 && F[k] <= 1.0;
                    }
                    if (!valid) continue;
                    int c = 0;
                    for (int k = 0; k < NCORNER; ++k) c |= (F[k] < 0.0) << k;
                    for (int i = 0; i < n_tri[c]; ++i, ++n) {
                        if (n >= cap) continue;
                        for (int j = 0; j < 3; ++j) {
                            int e = tri_edges[c][3 * i + j], lo, hi;
                            edge_corners(e, &lo, &hi);
                            int a = e / 4;
                            int64_t p[3];
                            for (int k = 0; k < 3; ++k) p[k] = g[k] + corner_coord(lo, k);
                            double te = F[lo] / (F[lo] - F[hi]);
                            if (vid) vid[3 * n + j] = 3 * (p[0] + (int64_t)G[0] * (p[1] + (int64_t)G[1] * p[2])) + a;
                            if (t) t[3 * n + j] = te;
                            if (pos)
                                for (int k = 0; k < 3; ++k)
                                    pos[9 * n + 3 * j + k] =
                                        origin[k] + ((double)p[k] + 0.5 + (k == a ? te : 0.0)) * vs;
                        }
                    }
                }
    }
    return n;
}

"""Pins of the oracle's marching cubes (Section 5: occupancy and counts,
prefix sum, polygonisation of the occupied cells).

The case table is derived in the oracle from a stated rule rather than
copied; these checks hold it to what a marching-cubes surface must be,
independently of how the table was built:
  * every case uses exactly the cube edges whose corners differ;
  * neighbouring cells cut their shared face the same way, in opposite
    directions (brute force over every pair of cases and every axis), and a
    patch's open border lies only on the cube's faces;
  * triangles face the positive (outside) side;
  * a linear field gives vertices exactly on its plane, and the mesh area
    equals the area of the plane clipped to the cells (closed form);
  * a sphere gives a closed, consistently oriented 2-manifold of Euler
    characteristic 2 whose vertices and volume lie within the
    interpolation bound of the sphere;
  * a chi voxel or an unallocated block removes exactly the cells that
    touch it.
"""

import itertools
import math

import numpy as np
import pytest

import oracle

CHI = oracle.CHI


@pytest.fixture(scope="module")
def table():
    oracle.build(force=False)
    return [oracle.mc_case(c) for c in range(256)]


def corner(k):
    return np.array([k & 1, (k >> 1) & 1, (k >> 2) & 1])


def edge_corners(e):
    """Cube edge 4a + m: along axis a, the other axes (increasing) at (m & 1, m >> 1)."""
    a, m = divmod(e, 4)
    other = [b for b in range(3) if b != a]
    lo = ((m & 1) << other[0]) | (((m >> 1) & 1) << other[1])
    return lo, lo | (1 << a)


def crossing_edges(c):
    out = set()
    for e in range(12):
        lo, hi = edge_corners(e)
        if ((c >> lo) & 1) != ((c >> hi) & 1):
            out.add(e)
    return out


def test_every_case_uses_exactly_its_crossing_edges(table):
    assert len(table[0]) == 0 and len(table[255]) == 0
    for c in range(256):
        used = set(table[c].ravel().tolist())
        assert used == crossing_edges(c), c
        for tri in table[c]:
            assert len(set(tri.tolist())) == 3, c


def test_unambiguous_classes_have_their_triangle_counts(table):
    # one corner cut off (or all but one): one triangle; two corners sharing
    # an edge: a quadrilateral; a whole face: a quadrilateral
    for c in range(256):
        n = bin(c).count("1")
        if n in (1, 7):
            assert len(table[c]) == 1, c
    for e in range(12):
        lo, hi = edge_corners(e)
        c = (1 << lo) | (1 << hi)
        assert len(table[c]) == 2 and len(table[255 ^ c]) == 2, c
    for a in range(3):
        for side in range(2):
            c = sum(1 << k for k in range(8) if corner(k)[a] == side)
            assert len(table[c]) == 2, c


def face_of_edge(e):
    """Faces (axis, side) that cube edge e lies on."""
    lo, _ = edge_corners(e)
    a = e // 4
    return {(b, int(corner(lo)[b])) for b in range(3) if b != a}


def boundary(tris):
    """Directed border edges of a triangle patch (edges used by one triangle)."""
    count = {}
    directed = []
    for t in tris:
        for i in range(3):
            u, v = int(t[i]), int(t[(i + 1) % 3])
            count[frozenset((u, v))] = count.get(frozenset((u, v)), 0) + 1
            directed.append((u, v))
    return [d for d in directed if count[frozenset(d)] == 1], count


def test_patch_border_lies_on_faces_and_interior_edges_pair_up(table):
    for c in range(256):
        border, count = boundary(table[c])
        assert max(count.values(), default=1) <= 2, c
        for u, v in border:
            assert face_of_edge(u) & face_of_edge(v), (c, u, v)


def shared_edge_map(a):
    """Cube edge on face x_a = 1 of a cell -> the same edge on face x_a = 0 of its +a neighbour."""
    out = {}
    for e in range(12):
        if e // 4 == a:
            continue
        lo, hi = edge_corners(e)
        if corner(lo)[a] == 1:
            lo2 = lo & ~(1 << a)
            for e2 in range(12):
                if edge_corners(e2)[0] == lo2 and e2 // 4 == e // 4:
                    out[e] = e2
    return out


def test_neighbouring_cells_cut_their_shared_face_alike(table):
    borders = [boundary(table[c])[0] for c in range(256)]
    for a in range(3):
        emap = shared_edge_map(a)
        face1 = [k for k in range(8) if corner(k)[a] == 1]
        for cA in range(256):
            on_face = [(u, v) for u, v in borders[cA] if (a, 1) in face_of_edge(u) & face_of_edge(v)]
            segA = {(emap[u], emap[v]) for u, v in on_face}
            for rest in range(16):
                cB = 0
                for k in face1:                      # B's face x_a = 0 carries A's x_a = 1 corners
                    cB |= ((cA >> k) & 1) << (k & ~(1 << a))
                free = [k for k in range(8) if corner(k)[a] == 1]
                for i, k in enumerate(free):
                    cB |= ((rest >> i) & 1) << k
                segB = {(u, v) for u, v in borders[cB] if (a, 0) in face_of_edge(u) & face_of_edge(v)}
                # same segments, opposite directions
                assert segB == {(v, u) for u, v in segA}, (a, cA, cB)


def trilinear_grad(vals, p):
    x, y, z = p
    v = lambda i, j, k: vals[i + 2 * j + 4 * k]  # noqa: E731
    gx = ((1 - y) * (1 - z) * (v(1, 0, 0) - v(0, 0, 0)) + y * (1 - z) * (v(1, 1, 0) - v(0, 1, 0)) +
          (1 - y) * z * (v(1, 0, 1) - v(0, 0, 1)) + y * z * (v(1, 1, 1) - v(0, 1, 1)))
    gy = ((1 - x) * (1 - z) * (v(0, 1, 0) - v(0, 0, 0)) + x * (1 - z) * (v(1, 1, 0) - v(1, 0, 0)) +
          (1 - x) * z * (v(0, 1, 1) - v(0, 0, 1)) + x * z * (v(1, 1, 1) - v(1, 0, 1)))
    gz = ((1 - x) * (1 - y) * (v(0, 0, 1) - v(0, 0, 0)) + x * (1 - y) * (v(1, 0, 1) - v(1, 0, 0)) +
          (1 - x) * y * (v(0, 1, 1) - v(0, 1, 0)) + x * y * (v(1, 1, 1) - v(1, 1, 0)))
    return np.array([gx, gy, gz])


def test_triangles_face_the_positive_side(table):
    # corners at -1 (inside) and +1: every vertex at its edge's midpoint, and
    # each triangle's winding normal has a positive component along the
    # gradient of the trilinear field at its centroid
    for c in range(1, 255):
        vals = [-1.0 if (c >> k) & 1 else 1.0 for k in range(8)]
        for tri in table[c]:
            P = [(corner(edge_corners(e)[0]) + corner(edge_corners(e)[1])) / 2.0 for e in tri]
            n = np.cross(P[1] - P[0], P[2] - P[0])
            g = trilinear_grad(vals, (P[0] + P[1] + P[2]) / 3.0)
            assert n @ g > 0, (c, tri)


# ---------------------------------------------------------------- volumes


def fill(vol, dims, vs, origin, sdf_fn, delta, skip=()):
    """Every block holding an in-band voxel centre gets sdf/delta, chi
    outside the band; values rounded to float32 (as a GPU volume holds them)."""
    l = np.arange(8)
    lz, ly, lx = np.meshgrid(l, l, l, indexing="ij")
    local = np.stack([lx.ravel(), ly.ravel(), lz.ravel()], -1)
    nb = [d // 8 for d in dims]
    for bz, by, bx in itertools.product(range(nb[2]), range(nb[1]), range(nb[0])):
        if (bx, by, bz) in skip:
            continue
        g = np.array([bx, by, bz]) * 8 + local
        sd = sdf_fn(np.asarray(origin) + (g + 0.5) * vs)
        if np.all(np.abs(sd) > delta):
            continue
        T = np.where(np.abs(sd) <= delta, sd / delta, CHI).astype(np.float32).astype(np.float64)
        vol.set_block((bx, by, bz), T)


def clipped_plane_area(n, h, lo, hi):
    """Area of {x : n.x = h} inside the box [lo, hi]: a large square on the
    plane clipped by the six half-spaces (Sutherland-Hodgman)."""
    n = n / np.linalg.norm(n)
    u = np.cross(n, [1.0, 0.0, 0.0] if abs(n[0]) < 0.9 else [0.0, 1.0, 0.0])
    u /= np.linalg.norm(u)
    w = np.cross(n, u)
    p0 = n * h
    L = 10.0 * float(np.max(np.abs(np.concatenate([lo, hi]))) + 1.0)
    poly = [p0 + L * (s * u + t * w) for s, t in ((-1, -1), (1, -1), (1, 1), (-1, 1))]
    for a in range(3):
        for sgn, bound in ((1.0, lo[a]), (-1.0, hi[a])):
            out = []
            for i in range(len(poly)):
                P, Q = poly[i], poly[(i + 1) % len(poly)]
                dp, dq = sgn * (P[a] - bound), sgn * (Q[a] - bound)
                if dp >= 0:
                    out.append(P)
                if (dp >= 0) != (dq >= 0):
                    out.append(P + (Q - P) * (dp / (dp - dq)))
            poly = out
    area = np.zeros(3)
    for i in range(1, len(poly) - 1):
        area += np.cross(poly[i] - poly[0], poly[i + 1] - poly[0])
    return 0.5 * float(np.linalg.norm(area))


def mesh_area(pos):
    return 0.5 * float(np.linalg.norm(np.cross(pos[:, 1] - pos[:, 0], pos[:, 2] - pos[:, 0]), axis=-1).sum())


@pytest.mark.parametrize("n,h", [((0.3, 0.5, 0.81), 0.2), ((0.0, 0.0, 1.0), 0.1003), ((-0.6, 0.2, 0.4), -0.05)])
def test_plane_vertices_on_the_plane_and_area_exact(n, h):
    dims, vs, origin = (40, 32, 48), 0.01, (-0.2, -0.15, -0.2)
    delta = 4 * vs
    nn = np.asarray(n) / np.linalg.norm(n)
    vol = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, 4096)
    fill(vol, dims, vs, origin, lambda x: x @ nn - h, delta)
    vid, t, pos = vol.marching_cubes()
    assert len(vid) > 500
    # the stored values are float32 roundings of a linear field: vertices lie
    # on the plane up to the float32 rounding of the values (|dF| <= 6e-8 in
    # delta units, moved along an edge whose |dF/dt| >= vs |n_a| / delta)
    resid = np.abs(pos.reshape(-1, 3) @ nn - h)
    assert resid.max() <= 1e-6 * vs
    lo = np.asarray(origin) + 0.5 * vs
    hi = np.asarray(origin) + (np.asarray(dims) - 0.5) * vs
    ref = clipped_plane_area(nn, h, lo, hi)
    assert abs(mesh_area(pos) - ref) <= 1e-5 * ref
    # every non-degenerate triangle faces +n
    nrm = np.cross(pos[:, 1] - pos[:, 0], pos[:, 2] - pos[:, 0])
    big = np.linalg.norm(nrm, axis=-1) > 1e-6 * vs * vs
    assert (nrm[big] @ nn > 0).all()


def test_plane_through_voxel_centres_keeps_its_area():
    # F = 0 exactly on a layer of voxel centres (counted outside): vertices
    # land on those centres and the area is still the clipped plane's
    dims, vs, origin = (24, 24, 24), 0.125, (0.0, 0.0, 0.0)
    vol = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, 512)
    zc = origin[2] + (10 + 0.5) * vs
    fill(vol, dims, vs, origin, lambda x: x[:, 2] - zc, 4 * vs)
    vid, t, pos = vol.marching_cubes()
    assert np.abs(pos[..., 2] - zc).max() == 0.0
    # F = 0 counts as outside: the crossings are the z edges from the layer
    # below (F < 0) to the zero layer, at t = 1
    vox, axis = vertex_voxels(vid.reshape(-1), dims)
    assert (axis == 2).all() and (vox[:, 2] == 9).all() and (t == 1.0).all()
    lo = np.asarray(origin) + 0.5 * vs
    hi = np.asarray(origin) + (np.asarray(dims) - 0.5) * vs
    ref = clipped_plane_area(np.array([0.0, 0.0, 1.0]), zc, lo, hi)
    assert abs(mesh_area(pos) - ref) <= 1e-12 * ref


def sphere_volume(dims=(48, 48, 48), vs=0.01, r=0.17, skip=()):
    origin = (-0.24, -0.24, -0.24)
    c = np.array([0.013, -0.007, 0.004])
    vol = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, 4096)
    fill(vol, dims, vs, origin, lambda x: np.linalg.norm(x - c, axis=-1) - r, 4 * vs, skip=skip)
    return vol, c, r, vs


def test_sphere_is_a_closed_oriented_manifold_near_the_sphere():
    vol, c, r, vs = sphere_volume()
    vid, t, pos = vol.marching_cubes()
    assert len(vid) > 5000
    assert ((t >= 0) & (t <= 1)).all()
    # each undirected edge in exactly two triangles, once in each direction
    directed = {}
    for tri in vid:
        for i in range(3):
            e = (int(tri[i]), int(tri[(i + 1) % 3]))
            directed[e] = directed.get(e, 0) + 1
    assert max(directed.values()) == 1
    for (u, v) in directed:
        assert (v, u) in directed
    V = len(np.unique(vid))
    E = len(directed) // 2
    assert V - E + len(vid) == 2
    # vertices within the linear-interpolation bound of the sphere: along an
    # edge of length h the secant zero of |x - c| - r is off by <= h^2 / (2 r)
    d = np.linalg.norm(pos.reshape(-1, 3) - c, axis=-1) - r
    assert np.abs(d).max() <= vs * vs / (2 * r) + 1e-6 * vs
    # outward: the winding normal points away from the centre
    nrm = np.cross(pos[:, 1] - pos[:, 0], pos[:, 2] - pos[:, 0])
    cen = pos.mean(1) - c
    assert ((nrm * cen).sum(-1) > 0).all()
    # enclosed volume (divergence theorem) against 4/3 pi r^3
    vol_mesh = float(np.einsum("ij,ij->i", pos[:, 0] - c, np.cross(pos[:, 1] - c, pos[:, 2] - c)).sum()) / 6.0
    assert abs(vol_mesh - 4.0 / 3.0 * math.pi * r ** 3) <= 0.01 * 4.0 / 3.0 * math.pi * r ** 3


def canonical(vid):
    """Triangles as rotation-normalised vertex-id triples, sorted."""
    k = np.argmin(vid, axis=1)
    rows = np.arange(len(vid))
    out = np.stack([vid[rows, k], vid[rows, (k + 1) % 3], vid[rows, (k + 2) % 3]], 1)
    return out[np.lexsort(out.T[::-1])]


def vertex_voxels(vid, G):
    g = vid // 3
    return np.stack([g % G[0], (g // G[0]) % G[1], g // (G[0] * G[1])], -1), vid % 3


def test_chi_voxel_and_missing_block_remove_exactly_their_cells():
    full, c, r, vs = sphere_volume()
    G = (48, 48, 48)
    base = canonical(full.marching_cubes()[0])
    # a chi voxel in the band: the 8 cells that have it as a corner vanish
    keys, T, P = full.export()
    b = int(np.argmax((np.abs(T) < 0.5).sum(1)))
    k = int(np.argmax(np.abs(T[b]) < 0.5))
    g = keys[b] * 8 + np.array([k % 8, (k // 8) % 8, k // 64])
    T2 = T[b].copy()
    T2[k] = CHI
    full.set_block(keys[b], T2)
    holed = canonical(full.marching_cubes()[0])
    base_set = set(map(tuple, base.tolist()))
    holed_set = set(map(tuple, holed.tolist()))
    assert holed_set < base_set
    removed = np.array(sorted(base_set - holed_set))
    # every removed triangle belongs to a cell with g as a corner: all its
    # vertices sit on edges starting within one voxel below g
    vox, _ = vertex_voxels(removed.reshape(-1), G)
    assert ((vox >= g - 1) & (vox <= g + 1)).all()
    assert len(removed) > 0
    # a missing block: no triangle has a vertex whose cell could touch it
    kb = tuple(int(x) for x in keys[len(keys) // 2])
    gone, _, _, _ = sphere_volume(skip=(kb,))
    vid_g = gone.marching_cubes()[0]
    vox, _ = vertex_voxels(vid_g.reshape(-1), G)
    inside = np.all((vox >= np.array(kb) * 8) & (vox < np.array(kb) * 8 + 8), axis=1)
    assert not inside.any()
    assert set(map(tuple, canonical(vid_g).tolist())) < base_set

"""Marching cubes of the HIP library against the oracle (needs an MI355X).

Both sides extract from the same stored values: the oracle's volume (an
analytic field, or frames the oracle fused) is rounded to the GPU's storage
type, written back into a fresh oracle volume and imported into the GPU
volume.  The triangle lists must then agree bit for bit in topology and
winding (vertex ids, triangles compared after rotating each to start at its
smallest id, then sorted), and the edge parameters t within the rounding of
one float32 division.
"""

import itertools

import numpy as np
import pytest
import torch

import oracle
from synthetic.configs import config_c2, config_c3, sequence_frame, small_orbit
from tests.parity import Kvec, oracle_volume_for

pytestmark = pytest.mark.gpu

CHI = oracle.CHI
T_TOL = 1e-6        # edge parameter t (one float32 division of float32 values)


@pytest.fixture(scope="module")
def tsdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd as m

    m.lib()
    oracle.build(force=False)
    return m


def canonical(vid, *per_vertex):
    """Rotate each triangle to start at its smallest id (winding kept), sort."""
    k = np.argmin(vid, axis=1)
    rows = np.arange(len(vid))
    rot = [np.stack([a[rows, k], a[rows, (k + 1) % 3], a[rows, (k + 2) % 3]], 1) for a in (vid,) + per_vertex]
    order = np.lexsort(rot[0].T[::-1])
    return [r[order] for r in rot]


def vertex_table(vid, t):
    """Sorted unique vertex ids and their per-vertex values (t [.., 3] or
    positions [.., 3, 3]); asserts every occurrence of a vertex carries the
    same value."""
    v = vid.reshape(-1)
    tt = t.reshape(len(v), -1)
    order = np.argsort(v, kind="stable")
    v, tt = v[order], tt[order]
    first = np.r_[True, v[1:] != v[:-1]]
    idx = np.cumsum(first) - 1
    u = v[first]
    tu = tt[first]
    assert np.array_equal(tt, tu[idx]), "a vertex carries two values"
    return u, tu


def compare_meshes(g, o, vs):
    gvid, gt, gxyz = g
    ovid, ot, opos = o
    assert len(gvid) == len(ovid), f"triangle counts differ: gpu {len(gvid)} oracle {len(ovid)}"
    if len(ovid) == 0:
        return dict(triangles=0)
    cg, = canonical(gvid)
    co, = canonical(ovid)
    assert np.array_equal(cg, co), "triangle lists differ"
    ug, tg = vertex_table(gvid, gt)
    uo, to = vertex_table(ovid, ot)
    assert np.array_equal(ug, uo)
    dt = np.abs(tg.astype(np.float64) - to)
    assert dt.max() <= T_TOL, dt.max()
    assert ((tg >= 0) & (tg <= 1)).all()
    stats = dict(triangles=len(gvid), vertices=len(ug), max_dt=float(dt.max()))
    if gxyz is not None:
        _, pg = vertex_table(gvid, gxyz)
        _, po = vertex_table(ovid, opos)
        dp = np.abs(pg.astype(np.float64) - po)
        bound = T_TOL * vs + 2.0 ** -23 * np.abs(po)
        assert (dp <= bound).all(), float((dp - bound).max())
        stats["max_dpos_vox"] = float(dp.max() / vs)
    return stats


def gpu_mesh(gv, with_xyz=True):
    vid, t, xyz = gv.extract_mesh(with_xyz=with_xyz)
    torch.cuda.synchronize()
    return vid.cpu().numpy(), t.cpu().numpy(), (xyz.cpu().numpy() if xyz is not None else None)


def analytic_blocks(dims, vs, origin, sdf_fn, delta, dtype, skip=(), chi_voxels=()):
    """keys [n,3] int32 and T [n,512] (float64 holding `dtype` values) of a
    truncated analytic distance field: every block with an in-band centre."""
    l = np.arange(8)
    lz, ly, lx = np.meshgrid(l, l, l, indexing="ij")
    local = np.stack([lx.ravel(), ly.ravel(), lz.ravel()], -1)
    nb = [d // 8 for d in dims]
    keys, Ts = [], []
    for bz, by, bx in itertools.product(range(nb[2]), range(nb[1]), range(nb[0])):
        if (bx, by, bz) in skip:
            continue
        g = np.array([bx, by, bz]) * 8 + local
        sd = sdf_fn(np.asarray(origin) + (g + 0.5) * vs)
        if np.all(np.abs(sd) > delta):
            continue
        T = np.where(np.abs(sd) <= delta, sd / delta, CHI)
        for cg in chi_voxels:
            hit = np.all(g == np.asarray(cg), axis=1)
            T[hit] = CHI
        keys.append((bx, by, bz))
        Ts.append(T.astype(dtype).astype(np.float64))
    return np.array(keys, np.int32).reshape(-1, 3), np.array(Ts).reshape(-1, 512)


def load_both(tsdf, dims, vs, origin, keys, T, storage=0, dense=True, capacity=1 << 14):
    grid_kw = dict(dims=dims, voxel_size=vs, origin=origin, trunc_voxels=4.0, capacity_blocks=capacity,
                   hash_slots=2 * capacity)
    ov = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, capacity)
    for k, t in zip(keys, T):
        ov.set_block(k, t)
    gv = tsdf.Volume(storage=storage, max_width=64, max_height=64, dense_index=1 if dense else 0, **grid_kw)
    if len(keys):
        P = np.full_like(T, 0.1)
        gv.import_blocks(torch.from_numpy(keys), torch.from_numpy(T), torch.from_numpy(P))
    return ov, gv


def sphere_and_plane(x, c=np.array([0.013, 0.021, -0.007]), r=0.13):
    return np.minimum(np.linalg.norm(x - c, axis=-1) - r, x[:, 1] + 0.1)


@pytest.mark.parametrize("storage,dense", [(0, True), (0, False), (1, True)])
def test_analytic_field_with_holes(tsdf, storage, dense):
    # a sphere resting on a plane that runs into the grid's last voxel layer
    # (cells there have corners outside the grid), one block left out and
    # one chi voxel in the band
    dims, vs, origin = (48, 40, 56), 0.008, (-0.19, -0.13, -0.22)
    dtype = np.float16 if storage == 1 else np.float32
    keys, T = analytic_blocks(dims, vs, origin, sphere_and_plane, 4 * vs, dtype, skip=((2, 1, 3),),
                              chi_voxels=((20, 14, 27),))
    ov, gv = load_both(tsdf, dims, vs, origin, keys, T, storage=storage, dense=dense)
    print(f"[mesh] analytic storage={storage} dense={dense}: {len(keys)} blocks", flush=True)
    st = compare_meshes(gpu_mesh(gv), ov.marching_cubes(), vs)
    print(f"[mesh] analytic storage={storage} dense={dense}", st, flush=True)
    assert st["triangles"] > 5000


def test_fused_orbit(tsdf):
    spec = small_orbit(width=96, height=72, n_frames=4, G=256, vs=0.008)
    ov0 = oracle_volume_for(spec)
    for k in range(4):
        d, p = sequence_frame(spec, k)
        ov0.integrate(d.numpy(), Kvec(spec.K), p)
    keys, T, _ = ov0.export()
    T = T.astype(np.float32).astype(np.float64)
    g = spec.grid
    ov, gv = load_both(tsdf, g.dims, g.voxel_size, g.origin, keys, T, capacity=g.capacity_blocks)
    st = compare_meshes(gpu_mesh(gv), ov.marching_cubes(), g.voxel_size)
    print("[mesh] fused orbit", st, flush=True)
    assert st["triangles"] > 1000


def test_empty_volume_and_capped_output(tsdf):
    dims, vs, origin = (32, 32, 32), 0.01, (-0.16, -0.16, -0.16)
    ov, gv = load_both(tsdf, dims, vs, origin, np.zeros((0, 3), np.int32), np.zeros((0, 512)))
    vid, t, xyz = gpu_mesh(gv)
    assert len(vid) == 0
    keys, T = analytic_blocks(dims, vs, origin, lambda x: np.linalg.norm(x, axis=-1) - 0.1, 4 * vs, np.float32)
    ov, gv = load_both(tsdf, dims, vs, origin, keys, T)
    full = gpu_mesh(gv)
    n = len(full[0])
    assert n > 100
    # a short output buffer: the count is the whole mesh, the first cap
    # triangles are those of the full call (same pool order), nothing beyond
    cap = n // 3
    dev = torch.device("cuda")
    vid = torch.full((cap + 5, 3), -7, dtype=torch.int64, device=dev)
    tt = torch.full((cap + 5, 3), -7.0, dtype=torch.float32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    work = gv.mesh_workspace()
    gv.extract_mesh_into(vid[:cap], tt[:cap], None, count, work)
    torch.cuda.synchronize()
    assert int(count.item()) == n
    assert np.array_equal(vid[:cap].cpu().numpy(), full[0][:cap])
    assert np.array_equal(tt[:cap].cpu().numpy(), full[1][:cap])
    assert (vid[cap:].cpu().numpy() == -7).all()


@pytest.mark.parametrize("cfg", ["c2", "c3"])
def test_benchmark_size_volumes(tsdf, cfg):
    # the first two frames of the 640x480 orbit (2048^3, 1 mm) and of the
    # 1280x960 hand sequence (4096^3, 0.15 mm), fused by the oracle
    spec = config_c2(n_frames=2) if cfg == "c2" else config_c3(n_frames=2)
    ov0 = oracle_volume_for(spec)
    ov0.set_threads(8)
    for k in range(2):
        d, p = sequence_frame(spec, k)
        print(f"[mesh] {spec.name} oracle frame {k}", flush=True)
        ov0.integrate(d.numpy(), Kvec(spec.K), p)
    keys, T, _ = ov0.export()
    del ov0
    T = T.astype(np.float32).astype(np.float64)
    g = spec.grid
    ov, gv = load_both(tsdf, g.dims, g.voxel_size, g.origin, keys, T, capacity=g.capacity_blocks)
    print(f"[mesh] {spec.name}: {len(keys)} blocks", flush=True)
    st = compare_meshes(gpu_mesh(gv), ov.marching_cubes(), g.voxel_size)
    print(f"[mesh] {spec.name}", st, flush=True)
    assert st["triangles"] > 10000

"""Batched multi-scene step (needs an MI355X).

Every scene of a batch must end bitwise identical to the same scene driven
through the single-volume calls (sorted block export, stats counters and the
raycast maps of every step), whatever the noise model, storage type, index
mode, graph capture or raycast group; one scene is also checked against the
oracle directly.  Scenes differ in grid, voxel size, frame size and frame
count, so steps leave some scenes out.
"""

import numpy as np
import pytest
import torch

import oracle
from synthetic.configs import sequence_frame, small_orbit
from tests.parity import Kvec, compare_raycast, compare_volumes, gpu_volume_for, oracle_volume_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tsdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd as m

    m.lib()
    return m


def scenes():
    return [small_orbit(width=80, height=60, n_frames=4, G=256, vs=0.008, seed=2),
            small_orbit(width=96, height=72, n_frames=3, G=192, vs=0.01, seed=5),
            small_orbit(width=64, height=40, n_frames=2, G=320, vs=0.006, seed=7)]


def sorted_export(vol):
    keys, T, P = vol.export()
    torch.cuda.synchronize()
    k = keys.cpu().numpy().astype(np.int64)
    order = np.lexsort((k[:, 0], k[:, 1], k[:, 2]))
    return k[order], T.cpu()[order], P.cpu()[order]


STAT_KEYS = ("allocated_blocks", "total_updates", "total_fresh_updates", "total_new_blocks",
             "total_candidates", "total_touched_blocks", "frames", "status_flags")


RULES = {0: {}, 1: dict(w=0.2), 2: dict(weight_kind=1, w_max=60000.0)}   # Algorithms 3, 1, 2


@pytest.mark.parametrize("noise,graph,storage,dense,group,rule,persistent", [
    ("quadratic", True, 0, True, 4, 0, False),
    ("constant", False, 0, False, 8, 0, False),
    ("quadratic", True, 1, True, 1, 0, False),
    ("mlp", True, 0, True, 16, 0, False),
    ("quadratic", True, 0, True, 4, 1, False),
    ("quadratic", False, 1, True, 8, 2, False),
    # the single cooperative launch
    ("quadratic", False, 0, True, 4, 0, True),
    ("mlp", False, 0, True, 2, 0, True),
    ("quadratic", False, 1, True, 8, 2, True),
])
def test_batch_equals_plain(tsdf, noise, graph, storage, dense, group, rule, persistent):
    specs = scenes()
    kind = dict(quadratic=tsdf.NOISE_QUADRATIC, constant=tsdf.NOISE_CONSTANT, mlp=tsdf.NOISE_MLP)[noise]
    coeff = 0.05 if noise == "constant" else 0.0015
    params = None
    if noise == "mlp":
        from paper_1311_7194_amd import mlp as M

        params = M.params_from_values(M.init_params(3))
    def mk(s):
        v = gpu_volume_for(s, storage=storage, dense_index=dense)
        v.set_update_rule(rule, **RULES[rule])
        return v

    batched = [mk(s) for s in specs]
    plain = [mk(s) for s in specs]
    b = tsdf.Batch(batched, [s.K for s in specs], graph=graph)
    b.set_persistent(persistent)
    b.set_raycast_group(group)
    for v in plain:
        v.set_raycast_group(group)
    steps = max(s.n_frames for s in specs)
    for t in range(steps):
        print(f"[batch] {noise} graph={graph} storage={storage} dense={dense} G={group} rule={rule} "
              f"persistent={persistent} step {t}",
              flush=True)
        depths, poses = [], []
        for s in specs:
            if t < s.n_frames:
                d, p = sequence_frame(s, t)
                depths.append(d.cuda().contiguous())
                poses.append(p)
            else:
                depths.append(None)
                poses.append(None)
        b.step(depths, poses, kind, coeff, params)
        for k, s in enumerate(specs):
            if depths[k] is None:
                continue
            plain[k].integrate(depths[k], s.K, poses[k], kind, coeff, params)
            vp, np_ = plain[k].raycast(s.K, poses[k])
            torch.cuda.synchronize()
            assert torch.equal(vp, b.vertex[k]), (t, k)
            assert torch.equal(np_, b.normal[k]), (t, k)
            assert int((vp[..., 3] > 0).sum()) > 0
    for k in range(len(specs)):
        bs, ps = batched[k].stats(), plain[k].stats()
        for key in STAT_KEYS:
            assert bs[key] == ps[key], (k, key, bs[key], ps[key])
        kb, Tb, Pb = sorted_export(batched[k])
        kp, Tp, Pp = sorted_export(plain[k])
        assert np.array_equal(kb, kp)
        assert torch.equal(Tb, Tp) and torch.equal(Pb, Pp)


def test_batch_scene_against_oracle(tsdf):
    """Scene 0 fused and raycast inside a graph-captured batch vs the oracle."""
    specs = scenes()
    vols = [gpu_volume_for(s) for s in specs]
    ovol = oracle_volume_for(specs[0])
    b = tsdf.Batch(vols, [s.K for s in specs], graph=True)
    for t in range(specs[0].n_frames):
        depths, poses = [], []
        for s in specs:
            if t < s.n_frames:
                d, p = sequence_frame(s, t)
                depths.append(d.cuda().contiguous())
                poses.append(p)
            else:
                depths.append(None)
                poses.append(None)
        b.step(depths, poses)
        d0, p0 = sequence_frame(specs[0], t)
        ovol.integrate(d0.numpy(), Kvec(specs[0].K), p0, oracle.NOISE_QUADRATIC, 0.0015)
    torch.cuda.synchronize()
    st = compare_volumes(vols[0], ovol)
    print("[batch] scene 0 volume vs oracle", st, flush=True)
    K = specs[0].K
    _, pose = sequence_frame(specs[0], specs[0].n_frames - 1)
    ov, on, ofl = ovol.raycast(Kvec(K), pose, K.width, K.height, n_threads=8)
    rs = compare_raycast(b.vertex[0].cpu().numpy(), b.normal[0].cpu().numpy(), ov, on, ofl, pose,
                         specs[0].grid.voxel_size)
    print("[batch] scene 0 raycast vs oracle", rs, flush=True)


def test_batch_autotune_and_rejections(tsdf):
    specs = scenes()
    vols = [gpu_volume_for(s) for s in specs]
    b = tsdf.Batch(vols, [s.K for s in specs], graph=True)
    depths, poses = [], []
    for s in specs:
        d, p = sequence_frame(s, 0)
        depths.append(d.cuda().contiguous())
        poses.append(p)
    b.step(depths, poses)
    ref = [v.clone() for v in b.vertex]
    g, ms = b.autotune_raycast(poses, reps=2)
    torch.cuda.synchronize()
    assert g in (1, 2, 4, 8, 16) and ms > 0 and b.raycast_group == g
    for k in range(len(specs)):
        assert torch.equal(ref[k], b.vertex[k])   # same pose, same volume: same maps
    # a volume twice, mixed storage types, or a non-orthonormal pose are refused
    with pytest.raises(tsdf.TsdfError):
        tsdf.Batch([vols[0], vols[0]], [specs[0].K, specs[0].K])
    with pytest.raises(tsdf.TsdfError):
        tsdf.Batch([vols[0], gpu_volume_for(specs[1], storage=1)], [specs[0].K, specs[1].K])
    bad = [p.copy() for p in poses]
    bad[1][0][0] = 2.0
    with pytest.raises(tsdf.TsdfError):
        b.step(depths, bad)


def test_fuse_grid_autotune_keeps_results(tsdf):
    # the fusion grid changes how candidates are spread over workgroups, not
    # the result: a batch tuned on warm-up frames, then reset, must end
    # bitwise equal to a batch with the default grid
    specs = scenes()
    frames = []
    for s in specs:
        frames.append([sequence_frame(s, t) for t in range(s.n_frames)])
    ends = []
    for tune in (False, True):
        vols = [gpu_volume_for(s) for s in specs]
        b = tsdf.Batch(vols, [s.K for s in specs], graph=True)
        if tune:
            d0 = [f[0][0].cuda().contiguous() for f in frames]
            p0 = [f[0][1] for f in frames]
            grid, ms = b.autotune_fuse(d0, p0, reps=1)
            torch.cuda.synchronize()
            print(f"[batch] fusion grid {grid} ({ms:.3f} ms per step)", flush=True)
            assert grid in (1280, 1920, 2560, 3840, 5120) and b.fuse_grid == grid and ms > 0
            for v in vols:
                v.reset()
            b.set_fuse_grid(1280 if grid != 1280 else 5120)   # a grid other than the default
        for t in range(max(s.n_frames for s in specs)):
            depths = [f[t][0].cuda().contiguous() if t < len(f) else None for f in frames]
            poses = [f[t][1] if t < len(f) else None for f in frames]
            b.step(depths, poses)
        torch.cuda.synchronize()
        ends.append(([sorted_export(v) for v in vols], [x.clone() for x in b.vertex],
                     [{k: v.stats()[k] for k in STAT_KEYS} for v in vols]))
    (ea, va, sa), (eb, vb, sb) = ends
    assert sa == sb
    for x, y in zip(ea, eb):
        assert np.array_equal(x[0], y[0]) and torch.equal(x[1], y[1]) and torch.equal(x[2], y[2])
    for x, y in zip(va, vb):
        assert torch.equal(x, y)
    with pytest.raises(tsdf.TsdfError):
        b.set_fuse_grid(0)

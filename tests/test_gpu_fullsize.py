"""Parity at the benchmark sizes (needs an MI355X).

The first frames of the c2 orbit (640x480 into 2048^3 at 1 mm, pool of 2^20
blocks), the c3 hand (1280x960 into 4096^3 at 0.15 mm) in FP32, and two
scenes of the c5 batch through the batched step, each in the launch
configuration the benchmark times (autotuned ray group, dense index).  The
oracle integrates the same frames; whole volumes are compared (block sets
bit-exact, values within tolerance) and the raycast is compared on a seeded
sample of pixels that the oracle marches one by one.  Algorithms 1 and 2 and
the eviction are checked on the c2 volume the same way, FP16 storage on c3.
"""

import numpy as np
import pytest
import torch

import oracle
from synthetic.configs import config_c2, config_c3, config_c5, sequence_frame
from tests.parity import (Kvec, camera_depth, compare_raycast, compare_volumes, fp16_bounds, gpu_blocks,
                          oracle_volume_for)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tsdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd as m

    m.lib()
    return m


def sample_pixels(K, n, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, K.width, n), rng.integers(0, K.height, n)], 1).astype(np.int32)


def check_sampled_raycast(ov, vert, nrm, K, pose, voxel, n=3000, seed=11):
    pix = sample_pixels(K, n, seed)
    ovv, onn, ofl = ov.raycast(Kvec(K), pose, K.width, K.height, pixels=pix, n_threads=8)
    idx = pix[:, 1] * K.width + pix[:, 0]
    rs = compare_raycast(vert.cpu().numpy(), nrm.cpu().numpy(), ovv, onn, ofl, pose, voxel, pixels=idx)
    return rs


# the first 20 frames of each sequence: the frames the benchmark times
@pytest.mark.parametrize("cfg,frames", [("c2", 20), ("c3", 20)])
def test_benchmark_size_sequence(tsdf, cfg, frames):
    spec = config_c2() if cfg == "c2" else config_c3()   # the defined 100- and 300-frame sequences
    K = spec.K
    gv = tsdf.Volume.from_grid(spec.grid, max_width=K.width, max_height=K.height)
    ov = oracle_volume_for(spec)
    ov.set_threads(8)
    for k in range(frames):
        d, pose = sequence_frame(spec, k)
        print(f"[full] {spec.name} frame {k}", flush=True)
        ost = ov.integrate(d.numpy(), Kvec(K), pose)
        gv.integrate(d.cuda(), K, pose)
        st = gv.stats()
        assert st["frame_updates"] == ost["updates"] and st["frame_new_blocks"] == ost["new_blocks"], (st, ost)
        assert st["status_flags"] == 0
    vs = compare_volumes(gv, ov)
    print(f"[full] {spec.name} volume", vs, flush=True)
    group, _ = gv.autotune_raycast(K, pose)
    vert, nrm = gv.raycast(K, pose)
    torch.cuda.synchronize()
    rs = check_sampled_raycast(ov, vert, nrm, K, pose, spec.grid.voxel_size)
    print(f"[full] {spec.name} raycast (G={group})", rs, flush=True)
    assert rs["hits"] > 100


def test_benchmark_size_batch(tsdf):
    """Scenes 0 (504^3, 320x240) and 11 (2336^3, 640x480) of the 16-scene batch,
    two steps through the graph-captured batched step."""
    specs = [config_c5(0, frame_limit=2), config_c5(11, frame_limit=2)]
    vols = [tsdf.Volume.from_grid(s.grid, max_width=s.K.width, max_height=s.K.height) for s in specs]
    b = tsdf.Batch(vols, [s.K for s in specs], graph=True)
    ovs = [oracle_volume_for(s) for s in specs]
    for k in range(2):
        frames = [sequence_frame(s, k) for s in specs]
        b.step([f[0].cuda().contiguous() for f in frames], [f[1] for f in frames])
        for s, ov, (d, p) in zip(specs, ovs, frames):
            ov.integrate(d.numpy(), Kvec(s.K), p)
    torch.cuda.synchronize()
    for i, (s, ov, gv) in enumerate(zip(specs, ovs, vols)):
        vs = compare_volumes(gv, ov)
        _, pose = sequence_frame(s, 1)
        rs = check_sampled_raycast(ov, b.vertex[i], b.normal[i], s.K, pose, s.grid.voxel_size, n=2000)
        print(f"[full] batch {s.name}", vs, rs, flush=True)
        assert rs["hits"] > 300


@pytest.mark.parametrize("rule,kw", [(oracle.RULE_RUNNING, dict(w=0.2)),
                                     (oracle.RULE_WEIGHTED, dict(w=1.0, w_max=8.0))], ids=["alg1", "alg2"])
def test_benchmark_size_update_rules(tsdf, rule, kw):
    """Algorithms 1 and 2 on the first two frames of the c2 orbit."""
    spec = config_c2(n_frames=2)
    K = spec.K
    gv = tsdf.Volume.from_grid(spec.grid, max_width=K.width, max_height=K.height)
    ov = oracle_volume_for(spec)
    gv.set_update_rule(rule, **kw)
    ov.set_rule(rule, **kw)
    for k in range(2):
        d, pose = sequence_frame(spec, k)
        print(f"[full] rule {rule} frame {k}", flush=True)
        ost = ov.integrate(d.numpy(), Kvec(K), pose)
        gv.integrate(d.cuda(), K, pose)
        st = gv.stats()
        assert st["frame_updates"] == ost["updates"] and st["frame_new_blocks"] == ost["new_blocks"], (st, ost)
    vs = compare_volumes(gv, ov)
    print(f"[full] rule {rule}", vs, flush=True)
    assert vs["live"] > 1000000


def test_benchmark_size_eviction(tsdf):
    """The eviction the benchmark times (blocks with x >= half the grid out)
    after two frames of the c2 orbit, then a third frame fused into the
    compacted volume."""
    spec = config_c2(n_frames=3)
    K = spec.K
    gv = tsdf.Volume.from_grid(spec.grid, max_width=K.width, max_height=K.height)
    ov = oracle_volume_for(spec)
    for k in range(2):
        d, pose = sequence_frame(spec, k)
        ov.integrate(d.numpy(), Kvec(K), pose)
        gv.integrate(d.cuda(), K, pose)
    nb = spec.grid.dims[0] // 8
    lo, hi = [0, 0, 0], [nb // 2 - 1, 1023, 1023]
    gk, gT, gP = gv.evict(lo, hi)
    ok_, oT, oP = ov.evict(lo, hi)
    print(f"[full] eviction: gpu {len(gk)} / oracle {len(ok_)} blocks out", flush=True)
    assert len(ok_) > 10000 and gv.stats()["allocated_blocks"] == ov.n_blocks > 10000
    a = oracle.sorted_blocks(gk.cpu().numpy(), gT.float().cpu().numpy().astype(np.float64),
                             gP.float().cpu().numpy().astype(np.float64))
    b = oracle.sorted_blocks(ok_, oT, oP)
    assert np.array_equal(a[0], b[0])
    olive, glive = np.abs(b[1]) <= 1, np.abs(a[1]) <= 1
    assert int((olive != glive).sum()) <= 1e-6 * olive.size      # the tolerance of compare_volumes
    live = olive & glive
    assert np.abs(a[1][live] - b[1][live]).max() <= 1e-5
    assert (np.abs(a[2][live] - b[2][live]) <= 1e-5 * np.maximum(b[2][live], 1e-30)).all()
    print("[full] kept", compare_volumes(gv, ov), flush=True)
    d, pose = sequence_frame(spec, 2)
    ost = ov.integrate(d.numpy(), Kvec(K), pose)
    gv.integrate(d.cuda(), K, pose)
    st = gv.stats()
    assert st["frame_updates"] == ost["updates"] and st["frame_new_blocks"] == ost["new_blocks"], (st, ost)
    print("[full] after a third frame", compare_volumes(gv, ov), flush=True)


def test_benchmark_size_fp16(tsdf):
    """FP16 storage on the first two frames of the c3 hand (4096^3, 1280x960),
    with the bounds of the small FP16 case: block set and chi status exact,
    T_hat and P_hat within the bounds derived from FP16 rounding for two
    updates, raycast depth within 0.1 voxel on the seeded pixels both sides
    hit."""
    spec = config_c3()   # the defined 300-frame sequence; its first two frames
    K = spec.K
    gv = tsdf.Volume.from_grid(spec.grid, storage=tsdf.F16, max_width=K.width, max_height=K.height)
    ov = oracle_volume_for(spec)
    for k in range(2):
        d, pose = sequence_frame(spec, k)
        print(f"[full] fp16 {spec.name} frame {k}", flush=True)
        ost = ov.integrate(d.numpy(), Kvec(K), pose)
        gv.integrate(d.cuda(), K, pose)
        st = gv.stats()
        assert st["frame_updates"] == ost["updates"] and st["frame_new_blocks"] == ost["new_blocks"], (st, ost)
    gk, gT, gP = gpu_blocks(gv)
    ok_, oT, oP = oracle.sorted_blocks(*ov.export())
    assert np.array_equal(gk, ok_)
    glive, olive = np.abs(gT) <= 1, np.abs(oT) <= 1
    assert np.array_equal(glive, olive)
    dT = np.abs(gT[olive] - oT[olive])
    rP = np.abs(gP[olive] - oP[olive]) / np.maximum(oP[olive], 1e-30)
    print(f"[full] fp16 volume: live {int(olive.sum())}, max dT {dT.max():.3g}, rms dT "
          f"{np.sqrt((dT ** 2).mean()):.3g}, max rel dP {rP.max():.3g}", flush=True)
    t_bound, p_bound = fp16_bounds(2)
    assert dT.max() <= t_bound + 1e-5 and rP.max() <= p_bound + 1e-5
    vert, _ = gv.raycast(K, pose)
    torch.cuda.synchronize()
    pix = sample_pixels(K, 6000, 13)                  # the hand covers about 8 % of the frame
    ovv, _, ofl = ov.raycast(Kvec(K), pose, K.width, K.height, pixels=pix, n_threads=8)
    g = vert.cpu().numpy().reshape(-1, 4).astype(np.float64)[pix[:, 1] * K.width + pix[:, 0]]
    ok = (ofl & (oracle.AMBIGUOUS | oracle.BISECT_INVALID | oracle.MARGINAL)) == 0
    both = (g[:, 3] > 0) & ((ofl & oracle.HIT) > 0) & ok
    mism = ((g[:, 3] > 0) != ((ofl & oracle.HIT) > 0)) & ok
    dz = np.abs(camera_depth(g[both], pose) - camera_depth(ovv[both], pose)) / spec.grid.voxel_size
    print(f"[full] fp16 raycast: {int(both.sum())} pixels, {int(mism.sum())} hit/miss differences, "
          f"max dz {dz.max():.3g} voxel", flush=True)
    assert both.sum() > 300 and mism.sum() <= 0.01 * len(pix) and dz.max() <= 0.1

"""Parity at the benchmark sizes (needs an MI355X).

The first frames of the c2 orbit (640x480 into 2048^3 at 1 mm, pool of 2^20
blocks), the c3 hand (1280x960 into 4096^3 at 0.15 mm) in FP32, and two
scenes of the c5 batch through the batched step, each in the launch
configuration the benchmark times (autotuned ray group, dense index).  The
oracle integrates the same frames; whole volumes are compared (block sets
bit-exact, values within tolerance) and the raycast is compared on a seeded
sample of pixels that the oracle marches one by one.
"""

import numpy as np
import pytest
import torch

import oracle
from synthetic.configs import config_c2, config_c3, config_c5, sequence_frame
from tests.parity import Kvec, compare_raycast, compare_volumes, oracle_volume_for

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


@pytest.mark.parametrize("cfg,frames", [("c2", 2), ("c3", 2)])
def test_benchmark_size_sequence(tsdf, cfg, frames):
    spec = config_c2(n_frames=frames) if cfg == "c2" else config_c3(n_frames=frames)
    K = spec.K
    gv = tsdf.Volume.from_grid(spec.grid, max_width=K.width, max_height=K.height)
    ov = oracle_volume_for(spec)
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

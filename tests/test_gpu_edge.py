"""Edge cases of the HIP path (needs an MI355X).

Frames without a single valid measurement, frames of one pixel and ragged
sizes, a camera inside an allocated block (the near-plane path of the
raycast), a wide truncation band seen from close by and at grazing angles
(candidate boxes reaching the camera and crossing the grid's faces), and
exhaustion of the block pool and of the per-frame candidate list (sticky
flags, TSDF_EFULL, recovery by reset).
"""

import numpy as np
import pytest
import torch

import oracle
from synthetic import Intrinsics, look_at, render_depth, sphere_scene
from synthetic.configs import config_c1, sequence_frame
from tests.parity import Kvec, compare_raycast, compare_volumes, gpu_volume_for, oracle_volume_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tsdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd as m

    m.lib()
    return m


def test_frame_without_measurements(tsdf):
    spec = config_c1()
    K = spec.K
    d = torch.zeros((K.height, K.width), dtype=torch.float32)
    d[0::4] = float("nan")
    d[1::4] = float("inf")
    d[2::4] = -1.0
    pose = spec.poses[0]
    gv = gpu_volume_for(spec)
    ov = oracle_volume_for(spec)
    gv.integrate(d.cuda(), K, pose)
    ost = ov.integrate(d.numpy(), Kvec(K), pose)
    st = gv.stats()
    assert ost["updates"] == 0 and st["frame_updates"] == 0 and st["allocated_blocks"] == 0
    assert st["status_flags"] == 0
    vert, nrm = gv.raycast(K, pose)
    torch.cuda.synchronize()
    assert not vert.any() and not nrm.any()


@pytest.mark.parametrize("wh", [(1, 1), (3, 2), (9, 7), (17, 13)])
def test_tiny_and_ragged_frames(tsdf, wh):
    """The c1 sphere seen through frames of a few pixels (partial tiles everywhere)."""
    w, h = wh
    spec = config_c1()
    f = 150.0 * w / 160.0 if w > 1 else 150.0
    K = Intrinsics(f, f, (w - 1) / 2.0, (h - 1) / 2.0, w, h)
    pose = spec.poses[0]
    d = render_depth(spec.scene, K, pose).float()
    gv = gpu_volume_for(spec, max_wh=(17, 13))
    ov = oracle_volume_for(spec)
    ost = ov.integrate(d.numpy(), Kvec(K), pose)
    gv.integrate(d.cuda(), K, pose)
    st = gv.stats()
    assert st["frame_updates"] == ost["updates"] and st["frame_new_blocks"] == ost["new_blocks"]
    if ost["updates"]:
        compare_volumes(gv, ov)
    vert, nrm = gv.raycast(K, pose)
    torch.cuda.synchronize()
    ovv, onn, ofl = ov.raycast(Kvec(K), pose, w, h)
    rs = compare_raycast(vert.cpu().numpy(), nrm.cpu().numpy(), ovv, onn, ofl, pose, spec.grid.voxel_size)
    print(f"[edge] {w}x{h}", st["frame_updates"], rs, flush=True)


def test_camera_inside_an_allocated_block(tsdf):
    """A camera 1.5 voxels in front of the fused sphere: the block around it is
    allocated, so rays start at the camera (near-plane path)."""
    spec = config_c1(noise=False)
    K0 = spec.K
    pose0 = spec.poses[0]
    gv = gpu_volume_for(spec)
    ov = oracle_volume_for(spec)
    views = [pose0, look_at((0.25, 0.1, 0.45), (0.0, 0.0, 1.0)), look_at((-0.25, -0.1, 0.45), (0.0, 0.0, 1.0))]
    for p in views:
        d = render_depth(spec.scene, K0, p).float()
        ov.integrate(d.numpy(), Kvec(K0), p)
        gv.integrate(d.cuda(), K0, p)
    compare_volumes(gv, ov)
    vs = spec.grid.voxel_size
    eye = (0.0, 0.0, 0.7 - 1.5 * vs)              # sphere front at z = 0.7
    pose = look_at(eye, (0.0, 0.0, 1.0), up=(0.0, -1.0, 0.0))
    # the camera's block must be allocated for this to test the near path
    keys, _, _ = ov.export()
    cb = np.floor((np.asarray(eye) - np.asarray(spec.grid.origin)) / vs).astype(int) // 8
    assert any((keys == cb).all(1))
    K = Intrinsics(60.0, 60.0, 31.5, 23.5, 64, 48)
    vert, nrm = gv.raycast(K, pose)
    torch.cuda.synchronize()
    ovv, onn, ofl = ov.raycast(Kvec(K), pose, K.width, K.height)
    rs = compare_raycast(vert.cpu().numpy(), nrm.cpu().numpy(), ovv, onn, ofl, pose, vs)
    print("[edge] camera inside a block", rs, flush=True)
    assert rs["hits"] > 100


def test_wide_band_near_and_grazing_views(tsdf):
    """A truncation band of 12 voxels seen from 2 cm in front of the sphere
    (frustum cells reaching back to the camera, D - delta < 0), from outside
    the grid at a grazing angle (cells crossing the grid's faces) and from a
    corner: the candidate boxes must still hold every block that receives a
    value, so the block sets and values equal the oracle's."""
    import dataclasses

    spec = config_c1(noise=False)
    spec = dataclasses.replace(spec, grid=dataclasses.replace(spec.grid, trunc_voxels=12.0))
    K = Intrinsics(55.0, 55.0, 31.7, 23.4, 64, 48)
    views = [look_at((0.0, 0.0, 0.68), (0.0, 0.0, 1.0), up=(0.0, -1.0, 0.0)),
             look_at((0.6, 0.05, 1.0), (-1.0, 0.0, 1.1)),
             look_at((0.3, 0.3, 0.62), (-0.1, -0.05, 1.1))]
    gv = gpu_volume_for(spec, max_wh=(64, 48))
    ov = oracle_volume_for(spec)
    for p in views:
        d = render_depth(spec.scene, K, p).float()
        ost = ov.integrate(d.numpy(), Kvec(K), p)
        gv.integrate(d.cuda(), K, p)
        st = gv.stats()
        assert st["frame_updates"] == ost["updates"] and st["frame_new_blocks"] == ost["new_blocks"]
        print("[edge] wide band view:", ost["updates"], "updates,", ost["new_blocks"], "new blocks", flush=True)
        assert ost["updates"] > 0
    compare_volumes(gv, ov)


def test_pool_exhaustion_is_sticky_until_reset(tsdf):
    from paper_1311_7194_amd import Volume

    spec = config_c1()
    g = spec.grid
    d, pose = sequence_frame(spec, 0)
    # a pool of 64 blocks; the candidate list keeps its full size
    gv = Volume(g.dims, g.voxel_size, g.origin, g.trunc_voxels, 64, 128, max_width=spec.K.width,
                max_height=spec.K.height, max_candidates=g.capacity_blocks)
    gv.integrate(d.cuda(), spec.K, pose)
    st = gv.stats()
    assert st["status_flags"] & tsdf.tsdf.FLAG_POOL_FULL
    assert st["allocated_blocks"] == 64
    with pytest.raises(tsdf.TsdfError) as e:
        gv.integrate(d.cuda(), spec.K, pose)
    assert e.value.status == tsdf.tsdf.EFULL
    gv.reset()
    st = gv.stats()
    assert st["status_flags"] == 0 and st["allocated_blocks"] == 0
    # a sparse frame (a 5x5 patch of pixels) fits again
    d2 = torch.zeros_like(d)
    d2[58:63, 78:83] = d[58:63, 78:83]
    gv.integrate(d2.cuda(), spec.K, pose)
    st = gv.stats()
    assert st["status_flags"] == 0 and 0 < st["allocated_blocks"] <= 64


def test_candidate_list_overflow_flag(tsdf):
    from paper_1311_7194_amd import Volume

    spec = config_c1()
    g = spec.grid
    d, pose = sequence_frame(spec, 0)
    gv = Volume(g.dims, g.voxel_size, g.origin, g.trunc_voxels, g.capacity_blocks, g.hash_slots,
                max_width=spec.K.width, max_height=spec.K.height, max_candidates=16)
    gv.integrate(d.cuda(), spec.K, pose)
    st = gv.stats()
    assert st["status_flags"] & tsdf.tsdf.FLAG_CAND_FULL

"""HIP library against the oracle, element by element (needs an MI355X).

Block sets must be bit-exact; T_hat within 1e-5 (delta units), P_hat within
1e-5 relative; raycast depth within 1e-3 voxel and normals within 1e-3 rad
on pixels both hit, with any hit/miss disagreement explained by an oracle
flag (ambiguous bracket, marginal crossing).
"""

import math

import numpy as np
import pytest
import torch

import oracle
from synthetic import Intrinsics, look_at
from synthetic.configs import config_c1, sequence_frame, small_orbit
from tests.parity import (Kvec, compare_raycast, compare_volumes, gpu_volume_for, oracle_volume_for)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tsdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd as m

    m.lib()
    return m


def run_both(spec, frames, q_hat=1e-4, storage=0, noise_kind=oracle.NOISE_QUADRATIC, coeff=0.0015):
    gv = gpu_volume_for(spec, storage=storage, q_hat=q_hat)
    ov = oracle_volume_for(spec, q_hat=q_hat)
    for k in frames:
        depth, pose = sequence_frame(spec, k)
        print(f"[parity] {spec.name} frame {k}", flush=True)
        ost = ov.integrate(depth.numpy(), Kvec(spec.K), pose, noise_kind, coeff)
        gv.integrate(depth.cuda(), spec.K, pose, noise_kind, coeff)
        gst = gv.stats()
        assert gst["frame_updates"] == ost["updates"], (gst, ost)
        assert gst["frame_new_blocks"] == ost["new_blocks"], (gst, ost)
        assert gst["status_flags"] == 0
    return gv, ov


def test_c1_single_frame_fusion_and_raycast(tsdf):
    spec = config_c1()
    gv, ov = run_both(spec, [0])
    st = compare_volumes(gv, ov)
    print("[parity] c1 volume", st, flush=True)
    depth, pose = sequence_frame(spec, 0)
    vert, nrm = gv.raycast(spec.K, pose)
    torch.cuda.synchronize()
    ovv, onn, ofl = ov.raycast(Kvec(spec.K), pose, spec.K.width, spec.K.height)
    rs = compare_raycast(vert.cpu().numpy(), nrm.cpu().numpy(), ovv, onn, ofl, pose, spec.grid.voxel_size)
    print("[parity] c1 raycast", rs, flush=True)
    assert rs["hits"] > 4000


def test_orbit_sequence_fusion_and_raycast(tsdf):
    """Six frames of a reduced orbit (ragged 100x75 frames, dropout, boxes)."""
    spec = small_orbit(width=100, height=75, n_frames=6, G=256, vs=0.008)
    gv, ov = run_both(spec, range(6))
    st = compare_volumes(gv, ov)
    print("[parity] orbit volume", st, flush=True)
    assert st["blocks"] > 300
    depth, pose = sequence_frame(spec, 3)
    vert, nrm = gv.raycast(spec.K, pose)
    torch.cuda.synchronize()
    ovv, onn, ofl = ov.raycast(Kvec(spec.K), pose, spec.K.width, spec.K.height, n_threads=8)
    rs = compare_raycast(vert.cpu().numpy(), nrm.cpu().numpy(), ovv, onn, ofl, pose, spec.grid.voxel_size)
    print("[parity] orbit raycast", rs, flush=True)


def test_constant_variance_zero_q(tsdf):
    spec = small_orbit(width=64, height=48, n_frames=4, G=128, vs=0.016)
    gv, ov = run_both(spec, range(4), q_hat=0.0, noise_kind=oracle.NOISE_CONSTANT, coeff=0.05)
    compare_volumes(gv, ov)


@pytest.mark.parametrize("group,dense,close", [(8, True, False), (1, True, False), (16, True, False),
                                               (4, False, False), (2, True, False), (4, True, True),
                                               (8, False, True)])
def test_raycast_of_imported_oracle_volume(tsdf, group, dense, close):
    """The oracle's volume copied into the GPU: raycasts must agree for every
    ray group size, with the dense index and through the hash alone, from a
    distant camera and from one close to the surfaces (blocks projecting to
    hundreds of pixels)."""
    spec = small_orbit(width=96, height=72, n_frames=3, G=256, vs=0.008)
    ov = oracle_volume_for(spec)
    for k in range(3):
        d, p = sequence_frame(spec, k)
        ov.integrate(d.numpy(), Kvec(spec.K), p)
    keys, T, P = ov.export()
    gv = gpu_volume_for(spec, max_wh=(128, 96), dense_index=dense)
    gv.set_raycast_group(group)
    gv.import_blocks(torch.from_numpy(keys), torch.from_numpy(T).float(), torch.from_numpy(P).float())
    K = Intrinsics(110.0, 110.0, 60.3, 40.7, 121, 83)   # another camera, ragged size
    pose = look_at((0.35, 0.35, -0.35) if close else (0.9, 0.6, -0.7), (0.0, 0.1, 0.0))
    vert, nrm = gv.raycast(K, pose)
    torch.cuda.synchronize()
    ovv, onn, ofl = ov.raycast(Kvec(K), pose, K.width, K.height, n_threads=8)
    rs = compare_raycast(vert.cpu().numpy(), nrm.cpu().numpy(), ovv, onn, ofl, pose, spec.grid.voxel_size)
    print(f"[parity] imported raycast G={group} dense={dense} close={close}", rs, flush=True)
    assert rs["hits"] > 1000


def test_raycast_bitwise_independent_of_group_and_index(tsdf):
    """Group size and index mode change the speed of the raycast, never its
    maps: every (group, index) pair gives bitwise the same vertex and normal
    maps, here with blocks close to the camera (large projected footprints)."""
    spec = small_orbit(width=96, height=72, n_frames=3, G=256, vs=0.008)
    ov = oracle_volume_for(spec)
    for k in range(3):
        d, p = sequence_frame(spec, k)
        ov.integrate(d.numpy(), Kvec(spec.K), p)
    keys, T, P = ov.export()
    K = Intrinsics(150.0, 150.0, 63.5, 47.5, 127, 95)
    poses = [look_at((0.9, 0.6, -0.7), (0.0, 0.1, 0.0)), look_at((0.35, 0.35, -0.35), (0.0, 0.1, 0.0))]
    # visible blocks must include both small projections (per-pixel spans) and
    # ones spanning over 256 pixels (per-tile spans)
    g = spec.grid
    corners = np.array([[dx, dy, dz] for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)], np.float64)
    box = np.asarray(g.origin) + (8.0 * keys[:, None, :] + 0.5 + 8.0 * corners[None]) * g.voxel_size
    small = large = 0
    for pose in poses:
        xc = (box - pose[:, 3]) @ pose[:, :3]
        front = (xc[..., 2] > 0.05).all(1)
        u = K.fx * xc[..., 0] / xc[..., 2] + K.cx
        w = K.fy * xc[..., 1] / xc[..., 2] + K.cy
        vis = front & (u.max(1) > 0) & (u.min(1) < K.width) & (w.max(1) > 0) & (w.min(1) < K.height)
        span = (u.max(1) - u.min(1) + 3) * (w.max(1) - w.min(1) + 3)
        small += int((vis & (span < 200)).sum())
        large += int((vis & (span > 300)).sum())
    assert small > 100 and large > 100, (small, large)
    ref = None
    for dense in (True, False):
        gv = gpu_volume_for(spec, max_wh=(128, 96), dense_index=dense)
        gv.import_blocks(torch.from_numpy(keys), torch.from_numpy(T).float(), torch.from_numpy(P).float())
        for group in (1, 2, 4, 8, 16):
            gv.set_raycast_group(group)
            maps = [gv.raycast(K, pose) for pose in poses]
            torch.cuda.synchronize()
            maps = [(v.cpu(), n.cpu()) for v, n in maps]
            if ref is None:
                ref = maps
                assert all(int((v[..., 3] > 0).sum()) > 300 for v, _ in maps)
            for (v, n), (rv, rn) in zip(maps, ref):
                assert torch.equal(v, rv) and torch.equal(n, rn), (group, dense)


def test_raycast_footprint_query(tsdf):
    """The instrumented raycast gives the same maps and counts each block its
    march reads once: at least one per hit ray's block, at most all blocks."""
    spec = small_orbit(width=96, height=72, n_frames=3, G=256, vs=0.008)
    gv = gpu_volume_for(spec)
    n0, _, _ = gv.raycast_footprint(spec.K, sequence_frame(spec, 0)[1])
    assert n0 == 0   # empty volume
    for k in range(3):
        d, p = sequence_frame(spec, k)
        gv.integrate(d.cuda(), spec.K, p)
    st = gv.stats()
    _, pose = sequence_frame(spec, 1)
    for group in (1, 4):
        gv.set_raycast_group(group)
        v1, n1 = gv.raycast(spec.K, pose)
        blocks, v2, n2 = gv.raycast_footprint(spec.K, pose)
        torch.cuda.synchronize()
        assert torch.equal(v1, v2) and torch.equal(n1, n2)
        assert 0 < blocks <= st["allocated_blocks"]
        # every hit vertex lies in (the stencil of) a block the march read
        hits = int((v1[..., 3] > 0).sum())
        print(f"[parity] footprint G={group}: {blocks} of {st['allocated_blocks']} blocks, {hits} hits", flush=True)
        assert hits > 0

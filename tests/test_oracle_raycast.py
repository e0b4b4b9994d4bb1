"""Pins of the oracle's raycast (Section 5) on analytically filled volumes.

  * trilinear sampling equals scipy's order-1 map_coordinates;
  * an affine distance field (a plane) is interpolated exactly, so the
    bisected root and the central-difference normal match the analytic
    ray/plane intersection to rounding;
  * a truncated sphere distance gives the analytic ray/sphere root within
    0.05 voxel at incidence below 60 degrees and the radial normal within
    1e-2 rad (check (d));
  * a fused noise-free sphere stays within the projective-measurement
    error of that root.
"""

import math

import numpy as np
import pytest
from scipy import ndimage

import oracle
from synthetic import Intrinsics, look_at
from synthetic.configs import config_c1, sequence_frame

CHI = oracle.CHI


def fill_analytic(vol, dims, vs, origin, sdf_fn, delta):
    """Allocate every block with an in-band voxel and store sdf/delta (chi outside)."""
    l = np.arange(8)
    lz, ly, lx = np.meshgrid(l, l, l, indexing="ij")
    local = np.stack([lx.ravel(), ly.ravel(), lz.ravel()], -1)
    nb = [d // 8 for d in dims]
    count = 0
    for bz in range(nb[2]):
        for by in range(nb[1]):
            for bx in range(nb[0]):
                g = np.array([bx, by, bz]) * 8 + local
                x = np.asarray(origin) + (g + 0.5) * vs
                sd = sdf_fn(x)
                if np.all(np.abs(sd) > delta):
                    continue
                T = np.where(np.abs(sd) <= delta, sd / delta, CHI)
                vol.set_block((bx, by, bz), T, np.full(512, 0.1))
                count += 1
    return count


def test_trilinear_matches_map_coordinates(oracle_lib):
    dims, vs, origin = (16, 16, 16), 0.01, (0.1, -0.2, 0.3)
    vol = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, 64)
    rng = np.random.default_rng(21)
    dense = rng.uniform(-0.99, 0.99, (16, 16, 16))  # [z, y, x]
    for bz in range(2):
        for by in range(2):
            for bx in range(2):
                blk = dense[8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8]
                vol.set_block((bx, by, bz), blk.reshape(512))
    pts = np.asarray(origin) + rng.uniform(0.5 * vs, 15.5 * vs, (500, 3))
    q = (pts - np.asarray(origin)) / vs - 0.5
    ref = ndimage.map_coordinates(dense, [q[:, 2], q[:, 1], q[:, 0]], order=1)
    got = np.array([vol.sample(p) for p in pts])
    np.testing.assert_allclose(got, ref, atol=1e-13)
    # voxel centres return the stored value; outside the centre hull is invalid
    assert vol.sample(np.asarray(origin) + np.array([3.5, 4.5, 5.5]) * vs) == pytest.approx(dense[5, 4, 3], abs=1e-12)
    assert vol.sample(np.asarray(origin) + np.array([0.2, 4.5, 5.5]) * vs) is None


def test_chi_or_empty_neighbour_invalidates(oracle_lib):
    dims, vs, origin = (16, 16, 16), 0.01, (0.0, 0.0, 0.0)
    vol = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, 64)
    T = np.zeros(512)
    T[0] = CHI
    vol.set_block((0, 0, 0), T)
    assert vol.sample(np.array([1.0, 1.0, 1.0]) * vs) is None     # stencil holds voxel 0 (chi)
    assert vol.sample(np.array([2.0, 2.0, 2.0]) * vs) == 0.0
    assert vol.sample(np.array([8.0, 2.0, 2.0]) * vs) is None     # reaches the empty block x=1


@pytest.mark.parametrize("seed", [0, 1])
def test_plane_volume_exact_root_and_normal(oracle_lib, seed):
    rng = np.random.default_rng(30 + seed)
    n = rng.normal(size=3)
    n[2] = -abs(n[2]) - 1.0
    n /= np.linalg.norm(n)
    centre = np.array([0.01, -0.02, 0.9])
    h = float(n @ centre)
    dims, vs = (48, 48, 48), 0.008
    origin = tuple(centre - 24 * vs)
    delta = 4 * vs
    vol = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, 1 << 12)
    fill_analytic(vol, dims, vs, origin, lambda x: x @ n - h, delta)
    K = Intrinsics(90.0, 90.0, 31.5, 23.5, 64, 48)
    pose = look_at((0.05, 0.03, 0.2), centre)
    vert, nrm, flags = vol.raycast((K.fx, K.fy, K.cx, K.cy), pose, K.width, K.height)
    hit = (flags & oracle.HIT) > 0
    assert hit.mean() > 0.5
    R, t = pose[:, :3], pose[:, 3]
    jj, ii = np.divmod(np.arange(K.width * K.height), K.width)
    dc = np.stack([(ii - K.cx) / K.fx, (jj - K.cy) / K.fy, np.ones(ii.size)], -1)
    dw = dc @ R.T
    D = (h - n @ t) / (dw @ n)   # camera depth of the plane along each pixel ray
    z = (vert[:, :3] - t) @ R[:, 2]
    np.testing.assert_allclose(z[hit], D[hit], atol=1e-6 * vs)
    np.testing.assert_allclose(nrm[hit, :3], np.broadcast_to(n, (hit.sum(), 3)), atol=1e-9)
    # every hit lies on the plane and is flagged neither ambiguous nor marginal
    assert np.all(flags[hit] == oracle.HIT)


def sphere_truth(K, pose, c, r):
    R, t = pose[:, :3], pose[:, 3]
    jj, ii = np.divmod(np.arange(K.width * K.height), K.width)
    dc = np.stack([(ii - K.cx) / K.fx, (jj - K.cy) / K.fy, np.ones(ii.size)], -1)
    dw = dc @ R.T
    oc = t - c
    a = (dw * dw).sum(-1)
    b = (dw * oc).sum(-1)
    disc = b * b - a * (oc @ oc - r * r)
    lam = np.where(disc >= 0, (-b - np.sqrt(np.maximum(disc, 0))) / a, np.nan)
    p = t + lam[:, None] * dw
    nrm = (p - c) / r
    cosi = -(dw / np.linalg.norm(dw, axis=1, keepdims=True) * nrm).sum(-1)
    return lam, p, nrm, cosi


def test_sphere_volume_matches_analytic_root(oracle_lib):
    c, r = np.array([0.0, 0.0, 1.0]), 0.3
    dims, vs, origin = (128, 128, 128), 0.005, (-0.32, -0.32, 0.68)
    delta = 4 * vs
    vol = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, 4096)
    fill_analytic(vol, dims, vs, origin, lambda x: np.linalg.norm(x - c, axis=-1) - r, delta)
    K = Intrinsics(150.0, 150.0, 80.0, 60.0, 160, 120)
    pose = look_at((0.1, -0.05, 0.0), (0.0, 0.0, 1.0))
    vert, nrm, flags = vol.raycast((K.fx, K.fy, K.cx, K.cy), pose, K.width, K.height, n_threads=4)
    lam, p, n_true, cosi = sphere_truth(K, pose, c, r)
    R, t = pose[:, :3], pose[:, 3]
    frontal = np.isfinite(lam) & (cosi > math.cos(math.radians(60)))
    hit = (flags & oracle.HIT) > 0
    assert hit[frontal].mean() > 0.995
    sel = frontal & hit
    z = (vert[:, :3] - t) @ R[:, 2]
    assert np.max(np.abs(z[sel] - lam[sel])) < 0.05 * vs
    ang = np.arccos(np.clip((nrm[sel, :3] * n_true[sel]).sum(-1), -1, 1))
    assert ang.max() < 1e-2
    # no hit off the sphere
    assert not np.any(hit & ~np.isfinite(lam))


def test_fused_sphere_within_projective_error(oracle_lib):
    """One noise-free sphere frame fused and raycast from the same pose: the
    surface lies within the pixel-quantisation error of the projective
    measurement (about a pixel footprint times tan(incidence))."""
    spec = config_c1(noise=False)
    depth, pose = sequence_frame(spec, 0)
    g = spec.grid
    vol = oracle.OracleVolume.from_grid(g, q_hat=0.0)
    K = spec.K
    vol.integrate(depth.numpy(), (K.fx, K.fy, K.cx, K.cy), pose)
    vert, nrm, flags = vol.raycast((K.fx, K.fy, K.cx, K.cy), pose, K.width, K.height)
    lam, p, n_true, cosi = sphere_truth(K, pose, np.array([0.0, 0.0, 1.0]), 0.3)
    hit = (flags & oracle.HIT) > 0
    sel = hit & np.isfinite(lam) & (cosi > math.cos(math.radians(45)))
    assert sel.sum() > 3000
    foot = lam / K.fx
    err = np.abs(vert[sel, 2] - lam[sel])
    assert np.all(err <= foot[sel] * np.tan(np.arccos(cosi[sel])) + 0.25 * g.voxel_size)

"""Pins of the ICP oracle (Section 6) against closed forms, invariants and
exactly solvable cases; no GPU."""

import math

import numpy as np
import pytest

from oracle import icp as O
from synthetic.scenes import Intrinsics, Scene, look_at, render_depth, render_model_maps

CORNER = Scene(planes=np.array([[0.0, 1.0, 0.0, 0.0],      # floor y = 0
                                [0.0, 0.0, 1.0, -0.8],     # wall z = -0.8
                                [1.0, 0.0, 0.0, -0.7]]))   # wall x = -0.7
K_SMALL = Intrinsics(120.0, 120.0, 47.5, 35.5, 96, 72)


def _pairs_on_planes(rng, n_per=200):
    """Points on three non-parallel planes with their unit normals."""
    normals = np.array([[0.0, 1.0, 0.0], [0.3, 0.1, 0.95], [0.9, -0.2, 0.3]])
    normals /= np.linalg.norm(normals, axis=1, keepdims=True)
    ps, ns = [], []
    for nrm in normals:
        a = np.cross(nrm, [1.0, 0.0, 0.0]) if abs(nrm[0]) < 0.9 else np.cross(nrm, [0.0, 1.0, 0.0])
        a /= np.linalg.norm(a)
        b = np.cross(nrm, a)
        uv = rng.uniform(-0.5, 0.5, (n_per, 2))
        ps.append(0.2 * nrm + uv[:, :1] * a + uv[:, 1:] * b + np.array([0.1, -0.3, 1.2]))
        ns.append(np.repeat(nrm[None], n_per, 0))
    return np.concatenate(ps), np.concatenate(ns)


def _solve(p, q, n, shrink, theta=-1.0):
    C, b, m, S, _ = O.normal_system(p, q, n, shrink)
    x, lam, keep = O.thresholded_solve(C, b, len(p), theta)
    r, t = x[:3], x[3:]
    if shrink:
        r = r / S
        t = t - np.cross(r, m)
    return r, t, (C, b, m, S, x)


@pytest.mark.parametrize("shrink", [False, True])
def test_pure_translation_is_recovered_exactly(shrink):
    # the linearised functional is exact for a translation: r = 0, t = t_true
    rng = np.random.default_rng(1)
    p, n = _pairs_on_planes(rng)
    t_true = np.array([0.004, -0.011, 0.007])
    r, t, _ = _solve(p, p + t_true, n, shrink)
    assert np.abs(r).max() < 1e-12
    assert np.abs(t - t_true).max() < 1e-12


def test_small_rotation_is_recovered_to_second_order():
    rng = np.random.default_rng(2)
    p, n = _pairs_on_planes(rng)
    r_true = np.array([2e-4, -1e-4, 3e-4])
    t_true = np.array([1e-3, 2e-3, -1e-3])
    q = p @ O.rotation_increment(r_true).T + t_true
    for shrink in (False, True):
        r, t, _ = _solve(p, q, n, shrink)
        assert np.abs(r - r_true).max() < 1e-7      # |r|^2 ~ 1e-7 rad
        assert np.abs(t - t_true).max() < 1e-6


def test_scaled_and_unscaled_solves_agree():
    # Unit-cube scaling is a change of variables: with no direction dropped
    # the back-substituted solution must equal the unscaled one.  The
    # relations as printed (r = S r^, t = t^ + r x m) do not have this property.
    rng = np.random.default_rng(3)
    p, n = _pairs_on_planes(rng)
    q = p + rng.normal(0, 2e-3, p.shape)
    r0, t0, _ = _solve(p, q, n, False)
    r1, t1, (C, b, m, S, x) = _solve(p, q, n, True)
    assert np.abs(r1 - r0).max() < 1e-10 * max(1.0, np.abs(r0).max()) + 1e-13
    assert np.abs(t1 - t0).max() < 1e-10 * max(1.0, np.abs(t0).max()) + 1e-13
    r_printed = S * x[:3]
    t_printed = x[3:] + np.cross(r_printed, m)
    assert np.abs(r_printed - r0).max() > 1e3 * np.abs(r1 - r0).max() + 1e-9
    assert np.abs(t_printed - t0).max() > 1e-6


def test_planar_scene_drops_unobservable_directions():
    # one plane z = 0: translation in the plane and rotation about its normal
    # have zero eigenvalues and are dropped; the offset along the normal stays
    rng = np.random.default_rng(4)
    p = np.concatenate([rng.uniform(-1, 1, (500, 2)), np.zeros((500, 1))], 1)
    n = np.repeat(np.array([[0.0, 0.0, 1.0]]), 500, 0)
    q = p + np.array([0.01, 0.02, 0.003])
    for shrink in (False, True):
        C, b, m, S, _ = O.normal_system(p, q, n, shrink)
        x, lam, keep = O.thresholded_solve(C, b, len(p), 0.005)
        assert keep.sum() == 3
        r, t = x[:3], x[3:]
        if shrink:
            r = r / S
            t = t - np.cross(r, m)
        assert np.abs(r).max() < 1e-12
        assert np.abs(t - [0.0, 0.0, 0.003]).max() < 1e-12


def test_threshold_is_per_pair():
    # lambda/N: duplicating every pair doubles C but keeps the decisions
    rng = np.random.default_rng(5)
    p, n = _pairs_on_planes(rng, 50)
    q = p + rng.normal(0, 1e-3, p.shape)
    C, b, *_ = O.normal_system(p, q, n, True)
    C2, b2, *_ = O.normal_system(np.concatenate([p, p]), np.concatenate([q, q]), np.concatenate([n, n]), True)
    lam = np.sort(np.linalg.eigvalsh(C)) / len(p)
    theta = float(0.5 * (lam[2] + lam[3]))   # a threshold between two eigenvalues
    x1, _, k1 = O.thresholded_solve(C, b, len(p), theta)
    x2, _, k2 = O.thresholded_solve(C2, b2, 2 * len(p), theta)
    assert (k1 == k2).all() and k1.sum() == 3
    assert np.abs(x1 - x2).max() < 1e-12


def test_rotation_increment():
    r = np.array([1e-6, 2e-6, -3e-6])
    R = O.rotation_increment(r)
    assert np.abs(R @ R.T - np.eye(3)).max() < 1e-15
    assert abs(np.linalg.det(R) - 1.0) < 1e-15
    small = np.array([[1.0, -r[2], r[1]], [r[2], 1.0, -r[0]], [-r[1], r[0], 1.0]])   # the paper's form
    assert np.abs(R - small).max() < 1e-11
    # order: rotations about x, then y, then z
    a = 0.3
    assert np.allclose(O.rotation_increment([a, 0, 0]) @ [0, 1, 0], [0, math.cos(a), math.sin(a)])
    Rb = O.rotation_increment([0.1, 0.2, 0.0])
    Rx = O.rotation_increment([0.1, 0, 0])
    Ry = O.rotation_increment([0, 0.2, 0])
    assert np.allclose(Rb, Ry @ Rx)


def test_live_normals_face_the_camera_and_are_exact_on_a_plane():
    K = K_SMALL
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    sc = Scene(planes=np.array([[0.0, 0.0, -1.0, -1.5]]))      # the plane z = 1.5 (solid beyond)
    D = render_depth(sc, K, pose).numpy().astype(np.float32)
    v, nrm, ok = O.live_points(D, K.as_tuple())
    assert ok[:-1, :-1].all() and not ok[-1].any() and not ok[:, -1].any()
    nn = nrm[ok] / np.linalg.norm(nrm[ok], axis=1, keepdims=True)
    assert np.abs(nn - [0.0, 0.0, -1.0]).max() < 1e-12


def test_identity_association():
    # live depth and model maps from the same pose: every live pixel with a
    # normal matches its own model pixel, and the update is ~0
    K = K_SMALL
    pose = look_at((0.3, 0.5, 0.4), (-0.3, 0.0, -0.4))
    D = render_depth(CORNER, K, pose).numpy().astype(np.float32)
    MV, MN = render_model_maps(CORNER, K, pose)
    res = O.icp_step(D, K.as_tuple(), MV.numpy(), MN.numpy(), pose, pose, O.IcpParams(dist_max=0.01, cos_min=0.9))
    _, _, ok = O.live_points(D, K.as_tuple())
    own = np.arange(K.width * K.height).reshape(K.height, K.width)
    m = res["match"]
    # away from the corner's edges (where the live normal straddles two planes)
    assert (m[m >= 0] == own[m >= 0]).all()
    assert res["N"] > 0.9 * ok.sum()
    assert np.abs(res["x"]).max() < 1e-5
    assert np.abs(res["pose"] - pose).max() < 1e-5


def test_converges_to_the_true_pose_on_a_corner():
    # three orthogonal planes fix all six degrees of freedom; from a pose
    # off by ~1 degree and ~1 cm the iteration returns to the truth
    K = Intrinsics(240.0, 240.0, 95.5, 71.5, 192, 144)
    true = look_at((0.3, 0.5, 0.4), (-0.3, 0.0, -0.4))
    D = render_depth(CORNER, K, true).numpy().astype(np.float32)
    MV, MN = render_model_maps(CORNER, K, true)
    est = true.copy()
    est[:, :3] = O.rotation_increment([0.01, -0.015, 0.012]) @ true[:, :3]
    est[:, 3] += [0.008, -0.006, 0.01]
    params = O.IcpParams(dist_max=0.05, cos_min=0.8)
    for _ in range(12):
        est = O.icp_step(D, K.as_tuple(), MV.numpy(), MN.numpy(), true, est, params)["pose"]
    assert np.abs(est[:, 3] - true[:, 3]).max() < 1e-5
    assert np.abs(est[:, :3] - true[:, :3]).max() < 1e-5


def test_no_pairs_leaves_the_pose():
    K = K_SMALL
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    D = np.zeros((K.height, K.width), np.float32)
    MV = np.zeros((K.height, K.width, 4), np.float32)
    res = O.icp_step(D, K.as_tuple(), MV, MV, pose, pose)
    assert res["N"] == 0 and (res["pose"] == pose).all()

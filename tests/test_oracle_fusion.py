"""Pins of the oracle's measurement, allocation and Kalman update.

  (a) analytic plane and sphere depth maps give the closed-form truncated
      distance (Eq. 1 with the projective measurement of Section 7.1);
  (b) Algorithm 3 reduces to the running mean with constant variance and
      Q = 0 (Eq. 9), to the inverse-variance mean with varying variance,
      and settles at the Riccati steady state with Q > 0;
  (c) the sparse volume equals a brute-force dense volume on tiny grids.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from synthetic import Intrinsics, look_at, plane_scene, render_depth, sphere_scene
from synthetic.configs import config_c1, sequence_frame, small_orbit
from tests.bruteforce import block_mask, dense_kalman, dense_measure, dense_to_blocks

CHI = oracle.CHI


def Kvec(K):
    return (K.fx, K.fy, K.cx, K.cy)


def voxel_centres(keys, vs, origin):
    """World centres [n,512,3] of the voxels of blocks (x-fastest order)."""
    l = np.arange(8)
    lz, ly, lx = np.meshgrid(l, l, l, indexing="ij")
    local = np.stack([lx.ravel(), ly.ravel(), lz.ravel()], -1)  # [512,3], x fastest
    g = keys[:, None, :] * 8 + local[None]
    return np.asarray(origin)[None, None] + (g + 0.5) * vs


# ----------------------------------------------------------------- (a) plane


def test_fronto_parallel_plane_closed_form(oracle_lib):
    """Plane z = z0 seen head-on: T_hat = (z0 - z)/delta at every in-band voxel.

    The grid sits wholly inside the view, so the in-band set is exactly the
    voxel layers with |z0 - z| <= delta (a count fixed by the geometry alone).
    """
    K = Intrinsics(100.0, 100.0, 100.0, 100.0, 200, 200)
    z0 = 1.0137
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    depth = render_depth(plane_scene((0, 0, -1), -z0), K, pose).numpy().astype(np.float32)
    assert np.all(depth == np.float32(z0))
    dims, vs, origin = (32, 32, 32), 0.01, (-0.16, -0.16, 0.84)
    vol = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, 4096)
    st = vol.integrate(depth, Kvec(K), pose, oracle.NOISE_CONSTANT, 0.25)
    keys, T, P = vol.export()
    x = voxel_centres(keys, vs, origin)
    delta = 4 * vs
    band = np.abs(np.float64(np.float32(z0)) - x[..., 2]) <= delta
    live = np.abs(T) <= 1
    assert np.array_equal(live, band)
    np.testing.assert_allclose(T[live], (np.float64(np.float32(z0)) - x[..., 2][live]) / delta, atol=1e-12)
    assert np.all(P[live] == 0.25)
    zs = origin[2] + (np.arange(32) + 0.5) * vs
    n_layers = int(np.sum(np.abs(np.float64(np.float32(z0)) - zs) <= delta))
    assert st["updates"] == n_layers * 32 * 32
    # every allocated block holds a live voxel (Fig. 4 caption rule)
    assert np.all(live.any(axis=1))


def projective_pixel(x, K, pose):
    """Pixel of world points through a 3x4 projection matrix K [R^T | -R^T t]."""
    R, t = pose[:, :3], pose[:, 3]
    Km = np.array([[K.fx, 0, K.cx], [0, K.fy, K.cy], [0, 0, 1.0]])
    Pm = Km @ np.hstack([R.T, (-R.T @ t)[:, None]])
    h = np.concatenate([x, np.ones(x.shape[:-1] + (1,))], -1) @ Pm.T
    z = h[..., 2]
    return h[..., 0] / z, h[..., 1] / z, z


@pytest.mark.parametrize("scene_kind", ["tilted-plane", "sphere"])
def test_projective_distance_general_pose(oracle_lib, scene_kind):
    """T_hat = (D(pixel) - z_cam)/delta with D the analytic surface depth.

    The pixel is found through a projection matrix (not the oracle's
    expression) and the depth from the closed-form ray/surface intersection
    evaluated here, so a transposed rotation, a wrong sign or a wrong pixel
    fails.
    """
    K = Intrinsics(120.0, 118.0, 63.5, 47.25, 128, 96)
    if scene_kind == "tilted-plane":
        n = np.array([0.3, 0.2, -1.0])
        n /= np.linalg.norm(n)
        h = float(n @ np.array([0.02, -0.01, 1.1]))
        scene = plane_scene(n, h)
    else:
        scene = sphere_scene((0.02, -0.01, 1.1), 0.25)
    pose = look_at((0.15, -0.1, 0.0), (0.02, -0.01, 1.1))
    depth = render_depth(scene, K, pose).numpy().astype(np.float32)
    dims, vs = (64, 64, 64), 0.008
    origin = (0.02 - 0.256, -0.01 - 0.256, 1.1 - 0.256)
    vol = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, 1 << 14)
    vol.integrate(depth, Kvec(K), pose, oracle.NOISE_CONSTANT, 1.0)
    keys, T, P = vol.export()
    x = voxel_centres(keys, vs, origin)
    live = np.abs(T) <= 1
    u, v, z = projective_pixel(x[live], K, pose)
    i, j = np.floor(u + 0.5).astype(int), np.floor(v + 0.5).astype(int)
    clear = (np.abs((u + 0.5) % 1 - 0.5) < 0.4999) & (np.abs((v + 0.5) % 1 - 0.5) < 0.4999)
    assert clear.mean() > 0.99
    # analytic depth at those pixels, evaluated here
    R, t = pose[:, :3], pose[:, 3]
    dc = np.stack([(i - K.cx) / K.fx, (j - K.cy) / K.fy, np.ones_like(u)], -1)
    dw = dc @ R.T
    if scene_kind == "tilted-plane":
        D = (h - n @ t) / (dw @ n)
    else:
        c, r = np.array([0.02, -0.01, 1.1]), 0.25
        oc = t - c
        a = (dw * dw).sum(-1)
        b = (dw * oc).sum(-1)
        D = (-b - np.sqrt(b * b - a * (oc @ oc - r * r))) / a
    assert np.all(np.abs(D - depth[j, i]) <= 2e-7 * D)
    expect = (depth[j, i].astype(np.float64) - z) / (4 * vs)
    np.testing.assert_allclose(T[live][clear], expect[clear], atol=1e-9)
    # the analytic surface depth itself lies within float32 rounding of it
    # (half an ulp of D ~ 1 m is 6e-8 m, i.e. 2e-6 delta here)
    np.testing.assert_allclose(T[live][clear], ((D - z) / (4 * vs))[clear], atol=4e-6)


def test_sphere_sign_agrees_with_true_sdf(oracle_lib):
    """Noise-free sphere (the 160x120 single-frame geometry): wherever the
    true signed distance exceeds the pixel footprint plus the obliquity
    slack, the fused value has its sign."""
    spec = config_c1(noise=False)
    depth, pose = sequence_frame(spec, 0)
    g = spec.grid
    vol = oracle.OracleVolume.from_grid(g, q_hat=0.0)
    vol.integrate(depth.numpy(), Kvec(spec.K), pose)
    keys, T, _ = vol.export()
    x = voxel_centres(keys, g.voxel_size, g.origin)
    live = np.abs(T) <= 1
    c = np.array([0.0, 0.0, 1.0])
    sdf = np.linalg.norm(x - c, axis=-1) - 0.3
    foot = x[..., 2] / spec.K.fx  # pixel footprint at the voxel depth
    decided = live & (np.abs(sdf) > 2 * foot)
    assert decided.sum() > 1000
    assert np.all(np.sign(T[decided]) == np.sign(sdf[decided]))
    # projective distance never understates the Euclidean one by more than a footprint
    assert np.all(np.abs(T[live]) * g.delta >= np.abs(sdf[live]) - 2 * foot[live])


# ----------------------------------------------------------- (b) Algorithm 3


def test_alg3_first_measurement_initialises(oracle_lib):
    assert oracle.alg3_step(CHI, 0.0, 0.3, 0.07, 1e-4) == (0.3, 0.07)
    # a chi measurement leaves the state alone
    assert oracle.alg3_step(0.2, 0.05, CHI, 0.07, 1e-4) == (0.2, 0.05)


def test_alg3_constant_variance_is_running_mean(oracle_lib):
    """Q = 0, p constant: T_n = mean of the measurements, P_n = p / n (Eq. 9)."""
    rng = np.random.default_rng(11)
    meas = rng.uniform(-0.9, 0.9, 200)
    T, P = CHI, 0.0
    for n, m in enumerate(meas, 1):
        T, P = oracle.alg3_step(T, P, m, 0.3, 0.0)
        assert abs(T - meas[:n].mean()) < 1e-12
        assert abs(P - 0.3 / n) < 1e-15 * n + 1e-15


def test_alg3_varying_variance_is_inverse_variance_mean(oracle_lib):
    """Q = 0: T = sum(T_k/p_k)/sum(1/p_k), P = 1/sum(1/p_k); the same as
    Algorithm 2 with w_k = 1/p_k and no cap."""
    rng = np.random.default_rng(12)
    meas = rng.uniform(-0.9, 0.9, 100)
    p = rng.uniform(0.01, 2.0, 100)
    T, P = CHI, 0.0
    T2, W2 = CHI, 0.0
    for m, pk in zip(meas, p):
        T, P = oracle.alg3_step(T, P, m, pk, 0.0)
        T2, W2 = oracle.alg2_step(T2, W2, m, 1.0 / pk, math.inf)
    w = 1.0 / p
    assert abs(T - (meas * w).sum() / w.sum()) < 1e-12
    assert abs(P - 1.0 / w.sum()) < 1e-14
    assert abs(T - T2) < 1e-12 and abs(1.0 / W2 - P) < 1e-14


def test_alg3_steady_state(oracle_lib):
    """Q > 0, constant p: P converges to the root of P^2 + Q P - Q p = 0."""
    q, p = 1e-4, 0.3
    T, P = CHI, 0.0
    for _ in range(5000):
        T, P = oracle.alg3_step(T, P, 0.1, p, q)
    Pss = (-q + math.sqrt(q * q + 4 * q * p)) / 2
    assert abs(P - Pss) < 1e-12
    assert abs(T - 0.1) < 1e-12


def test_alg1_and_alg2_rules(oracle_lib):
    assert oracle.alg1_step(CHI, 0.4, 0.1) == 0.4
    assert abs(oracle.alg1_step(0.4, 0.0, 0.25) - 0.3) < 1e-15
    T, W = oracle.alg2_step(CHI, 0.0, 0.5, 2.0, 10.0)
    assert (T, W) == (0.5, 2.0)
    T, W = oracle.alg2_step(0.5, 9.0, -0.5, 3.0, 10.0)
    assert abs(T - 0.25) < 1e-15 and W == 10.0


def test_eq9_monte_carlo_variance(oracle_lib):
    """Averaging N normal deviates with Algorithm 3 (Q = 0) leaves variance sigma^2/N."""
    rng = np.random.default_rng(13)
    sigma, N, trials = 0.1, 16, 4000
    final = np.empty(trials)
    for k in range(trials):
        T, P = CHI, 0.0
        for m in rng.normal(0.0, sigma, N):
            T, P = oracle.alg3_step(T, P, m, sigma * sigma, 0.0)
        final[k] = T
    ratio = final.var() / (sigma * sigma / N)
    assert 0.9 < ratio < 1.1  # 4000 trials: standard error of the ratio ~0.022


def test_kalman_resists_growing_variance(oracle_lib):
    """Fig. 11 setting: measurement spread grows steadily; with parameters
    giving both filters the same smoothing at the start, the Kalman estimate
    (which knows p_k) ends closer to the truth than a constant-weight
    update."""
    rng = np.random.default_rng(14)
    n = 400
    sig = np.linspace(0.02, 0.4, n)
    errs_k, errs_w = [], []
    for trial in range(200):
        m = rng.normal(0.0, sig)
        Tk_, Pk_ = CHI, 0.0
        Tw = CHI
        q = 1e-5
        # steady-state Kalman gain at the starting variance sets the constant weight
        Pss = (-q + math.sqrt(q * q + 4 * q * sig[0] ** 2)) / 2
        w = (Pss + q) / (Pss + q + sig[0] ** 2)
        for k in range(n):
            Tk_, Pk_ = oracle.alg3_step(Tk_, Pk_, m[k], sig[k] ** 2, q)
            Tw = oracle.alg1_step(Tw, m[k], w)
        errs_k.append(Tk_ ** 2)
        errs_w.append(Tw ** 2)
    assert np.mean(errs_k) < 0.5 * np.mean(errs_w)


def test_volume_running_mean_on_plane_sequence(oracle_lib):
    """Constant-variance plane sequence with Q = 0: every voxel in band on all
    frames ends at the mean of its measurements and P = p/N."""
    K = Intrinsics(100.0, 100.0, 100.0, 100.0, 200, 200)
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    dims, vs, origin = (32, 32, 32), 0.01, (-0.16, -0.16, 0.84)
    vol = oracle.OracleVolume(dims, vs, origin, 4.0, 0.0, 4096)
    rng = np.random.default_rng(15)
    offs = rng.uniform(-0.003, 0.003, 12)
    zs = []
    for o in offs:
        z = np.float32(1.0 + o)
        zs.append(np.float64(z))
        depth = np.full((200, 200), z, np.float32)
        vol.integrate(depth, Kvec(K), pose, oracle.NOISE_CONSTANT, 0.2)
    keys, T, P = vol.export()
    x = voxel_centres(keys, vs, origin)[..., 2]
    always = np.ones_like(x, bool)
    for z in zs:
        always &= np.abs(z - x) <= 0.04
    assert always.sum() > 1000
    expect = (np.mean(zs) - x) / 0.04
    np.testing.assert_allclose(T[always], expect[always], atol=1e-12)
    np.testing.assert_allclose(P[always], 0.2 / len(zs), rtol=1e-12)


# -------------------------------------------------- (c) sparse == dense


def run_dense(spec, frames, q_hat, noise_coeff=0.0015):
    g = spec.grid
    Gx, Gy, Gz = g.dims
    T = np.full((Gz, Gy, Gx), CHI)
    P = np.zeros((Gz, Gy, Gx))
    alloc = np.zeros((Gz // 8, Gy // 8, Gx // 8), bool)
    for depth, pose in frames:
        valid, s, i, j = dense_measure(g.dims, g.voxel_size, g.origin, g.delta, depth, Kvec(spec.K), pose)
        D = depth[j, i].astype(np.float64)
        sigma = noise_coeff * D * D
        pk = (sigma * sigma) / (g.delta * g.delta)
        T, P = dense_kalman(T, P, valid, np.where(valid, s / g.delta, CHI), pk, q_hat)
        alloc |= block_mask(valid)
    return dense_to_blocks(T, P, alloc)


def compare_sparse_dense(vol, dense):
    keys, T, P = oracle.sorted_blocks(*vol.export())
    dk, dT, dP = oracle.sorted_blocks(*dense)
    assert np.array_equal(keys, dk)
    assert np.array_equal(np.abs(T) > 1, np.abs(dT) > 1)
    live = np.abs(T) <= 1
    np.testing.assert_allclose(T[live], dT[live], atol=1e-12)
    np.testing.assert_allclose(P[live], dP[live], rtol=1e-12)


def test_sparse_equals_dense_single_sphere_frame(oracle_lib):
    """The 160x120 sphere frame on its full 128^3 grid (2.1 M voxels)."""
    spec = config_c1()
    depth, pose = sequence_frame(spec, 0)
    depth = depth.numpy()
    vol = oracle.OracleVolume.from_grid(spec.grid, q_hat=1e-4)
    st = vol.integrate(depth, Kvec(spec.K), pose)
    dense = run_dense(spec, [(depth, pose)], 1e-4)
    compare_sparse_dense(vol, dense)
    assert st["updates"] == int((np.abs(dense[1]) <= 1).sum())
    assert st["new_blocks"] == len(dense[0])


def test_sparse_equals_dense_orbit_sequence(oracle_lib):
    """Four frames of a scaled-down orbit (boxes, spheres, ground, dropout)."""
    spec = small_orbit(width=64, height=48, n_frames=4, G=96, vs=0.02)
    frames = [tuple(x if i else x.numpy() for i, x in enumerate(sequence_frame(spec, k)))
              for k in range(spec.n_frames)]
    vol = oracle.OracleVolume.from_grid(spec.grid, q_hat=1e-4)
    for d, p in frames:
        vol.integrate(d, Kvec(spec.K), p)
    dense = run_dense(spec, frames, 1e-4)
    assert len(dense[0]) > 50
    compare_sparse_dense(vol, dense)


def test_threaded_integration_equals_serial(oracle_lib):
    """Rows of pixels on several threads give the same blocks, values and
    counts as the serial loop (only the allocation order may differ)."""
    spec = small_orbit(width=64, height=48, n_frames=3, G=96, vs=0.02)
    vols = []
    stats = []
    for threads in (1, 4):
        vol = oracle.OracleVolume.from_grid(spec.grid, q_hat=1e-4)
        vol.set_threads(threads)
        st = []
        for k in range(spec.n_frames):
            d, p = sequence_frame(spec, k)
            st.append(vol.integrate(d.numpy(), Kvec(spec.K), p))
        vols.append(oracle.sorted_blocks(*vol.export()))
        stats.append(st)
    assert stats[0] == stats[1]
    for a, b in zip(*vols):
        assert np.array_equal(a, b)
    with pytest.raises(ValueError):
        oracle.OracleVolume.from_grid(spec.grid).set_threads(0)


def test_capacity_exhaustion_reports_full(oracle_lib):
    spec = config_c1()
    depth, pose = sequence_frame(spec, 0)
    for threads in (1, 4):
        vol = oracle.OracleVolume.from_grid(spec.grid, capacity_blocks=10)
        vol.set_threads(threads)
        with pytest.raises(RuntimeError):
            vol.integrate(depth.numpy(), Kvec(spec.K), pose)
        assert vol.n_blocks == 10


def test_memory_formula(oracle_lib):
    """Block store bytes = (bytes per T + per P) * 512 * blocks (Fig. 6 caption
    with the variance stored beside the distance)."""
    spec = config_c1()
    depth, pose = sequence_frame(spec, 0)
    vol = oracle.OracleVolume.from_grid(spec.grid)
    vol.integrate(depth.numpy(), Kvec(spec.K), pose)
    keys, T, P = vol.export()
    assert T.nbytes + P.nbytes == 2 * 8 * 512 * vol.n_blocks

"""Pins of the oracle's measurement variance and of the learned model's
training update, against numbers worked out by hand.

  - The quadratic model (Section 7.1, Kalman paragraph: the deviation grows
    with the square of depth, so the variance with its fourth power) with the
    synthetic sensor's sigma = 0.0015 D^2: a first measurement stores
    P_hat = (0.0015 D^2)^2 / delta^2.  At D = 1 m and delta = 20 mm that is
    0.005625; at D = 2 m it is 0.09.  Using the voxel's camera depth for D,
    sigma for sigma^2 or delta for delta^2 gives other numbers.
  - The learned model's variance is exp(s) / delta^2 clamped to
    [p_q e^-4, p_q e^4] around the quadratic p_q, which also stands in where
    the features are undefined.  With the last layer's weights at zero the
    network outputs s = b3 exactly, so both clamps and the pass-through are
    checked against literal values.
  - Adam: two steps on one parameter, worked out by hand, and the closed form
    for a constant gradient (bias correction makes every step lr g / (|g| + eps)).
"""

import math

import numpy as np
import pytest

import oracle
from oracle.adam import adam_step
from synthetic import Intrinsics, plane_scene, render_depth

OFF_W3, OFF_B3 = 1216, 1248


def head_on_plane(z0, K):
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    depth = render_depth(plane_scene((0, 0, -1), -z0), K, pose).numpy().astype(np.float32)
    assert np.all(depth == np.float32(z0))
    return depth, pose


@pytest.mark.parametrize("z0,expect", [(1.0, 0.005625), (2.0, 0.09)])
def test_quadratic_variance_first_measurement(oracle_lib, z0, expect):
    """(0.0015 * 1^2 / 0.02)^2 = 0.075^2 = 0.005625; (0.0015 * 4 / 0.02)^2 = 0.3^2 = 0.09."""
    K = Intrinsics(100.0, 100.0, 100.0, 100.0, 200, 200)
    depth, pose = head_on_plane(z0, K)
    vs = 0.005   # delta = 4 voxels = 20 mm
    vol = oracle.OracleVolume((32, 32, 32), vs, (-0.08, -0.08, z0 - 0.08), 4.0, 1e-4, 4096)
    st = vol.integrate(depth, (K.fx, K.fy, K.cx, K.cy), pose, oracle.NOISE_QUADRATIC, 0.0015)
    _, T, P = vol.export()
    live = np.abs(T) <= 1
    # voxel centres at z0 - 17.5 mm .. z0 + 17.5 mm (8 layers), so a variance
    # taken from the voxel's own depth would vary across it
    assert st["updates"] == 8 * 32 * 32 and live.sum() == st["updates"]
    np.testing.assert_allclose(P[live], expect, rtol=1e-12)


def test_quadratic_variance_second_measurement(oracle_lib):
    """The same plane twice at 1 m, Q_hat = 1e-4: the prediction gives
    P' = 0.005725, the gain 0.005725 / 0.01135 and the variance
    (1 - gain) P' = 0.005725 * 0.005625 / 0.01135."""
    K = Intrinsics(100.0, 100.0, 100.0, 100.0, 200, 200)
    depth, pose = head_on_plane(1.0, K)
    vol = oracle.OracleVolume((32, 32, 32), 0.005, (-0.08, -0.08, 0.92), 4.0, 1e-4, 4096)
    for _ in range(2):
        vol.integrate(depth, (K.fx, K.fy, K.cx, K.cy), pose, oracle.NOISE_QUADRATIC, 0.0015)
    _, T, P = vol.export()
    live = np.abs(T) <= 1
    np.testing.assert_allclose(P[live], 0.005725 * 0.005625 / 0.01135, rtol=1e-12)


def plane_with_hole():
    K = Intrinsics(50.0, 50.0, 20.0, 15.0, 40, 30)
    depth, _ = head_on_plane(1.0, K)
    depth[10:15, 15:21] = 0.0
    # features exist where the pixel is off the image border and it and its
    # four neighbours have a depth
    ok = depth > 0
    feat = np.zeros_like(ok)
    feat[1:-1, 1:-1] = ok[1:-1, 1:-1] & ok[:-2, 1:-1] & ok[2:, 1:-1] & ok[1:-1, :-2] & ok[1:-1, 2:]
    return depth, K, ok, feat


@pytest.mark.parametrize("b3,expect", [
    (-8.0, 0.005625 * math.exp(4.0)),     # exp(-8)/4e-4 = 0.839 > p_q e^4 = 0.307: upper clamp
    (-18.0, 0.005625 * math.exp(-4.0)),   # exp(-18)/4e-4 = 3.8e-5 < p_q e^-4 = 1.03e-4: lower clamp
    (-12.5, math.exp(-12.5) / 4e-4),      # 0.00932, inside the band: passed through
])
def test_learned_variance_clamp_and_fallback(oracle_lib, b3, expect):
    depth, K, ok, feat = plane_with_hole()
    params = np.zeros(oracle.MLP_PARAMS)
    params[OFF_B3] = b3   # exact in bfloat16
    p = oracle.mlp_variance(depth, (K.fx, K.fy, K.cx, K.cy), params, delta=0.02).reshape(depth.shape)
    assert feat.sum() > 800 and (ok & ~feat).sum() > 100
    np.testing.assert_allclose(p[feat], expect, rtol=1e-12)
    # measured pixels without features keep the quadratic variance
    np.testing.assert_allclose(p[ok & ~feat], 0.005625, rtol=1e-12)


def test_adam_two_steps_by_hand():
    """w = 1, gradients 0.5 then -0.25, lr 1e-3, betas 0.9 / 0.999, eps 1e-8.
    Step 1: m = 0.05, v = 0.00025, m_hat = 0.5, v_hat = 0.25,
            w = 1 - 1e-3 * 0.5 / (0.5 + 1e-8) = 0.99900000002.
    Step 2: m = 0.045 - 0.025 = 0.02, v = 0.00024975 + 0.0000625 = 0.00031225,
            m_hat = 0.02 / 0.19 = 0.105263157894737,
            v_hat = 0.00031225 / 0.001999 = 0.156203101550775,
            w = 0.998733662987078."""
    w, m, v = adam_step(np.array([1.0]), np.zeros(1), np.zeros(1), np.array([0.5]), 1)
    assert m[0] == pytest.approx(0.05, rel=1e-15) and v[0] == pytest.approx(0.00025, rel=1e-12)
    assert w[0] == pytest.approx(0.99900000002, rel=1e-15)
    w, m, v = adam_step(w, m, v, np.array([-0.25]), 2)
    assert m[0] == pytest.approx(0.02, rel=1e-12) and v[0] == pytest.approx(0.00031225, rel=1e-12)
    assert w[0] == pytest.approx(0.9987336629870785, rel=1e-15)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the corrected moments are exactly g and g^2,
    so every step moves each weight by lr * g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w0 = np.array([0.5, -1.0, 2.0, 0.25])
    w, m, v = w0.copy(), np.zeros(4), np.zeros(4)
    for t in range(1, 11):
        w, m, v = adam_step(w, m, v, g, t)
    np.testing.assert_allclose(w, w0 - 10 * 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    with pytest.raises(ValueError):
        adam_step(w, m, v, g, 0)

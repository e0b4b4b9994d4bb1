"""Pins of the oracle's Algorithms 1 and 2 as volume update rules.

A fronto-parallel plane moving in depth gives every voxel in band a known
sequence of measurements, so each rule's result has a closed form:
  * Algorithm 1 with constant w is an exponentially weighted mean;
  * Algorithm 2 with constant w and no cap is the plain mean (W = N w);
  * Algorithm 2 whose cap equals one weight is Algorithm 1 with w = 1/2;
  * Algorithm 2 with inverse-variance weights and no cap is Algorithm 3 with
    Q = 0 (T equal, P = 1/W), even when the variance changes per frame.
"""

import math

import numpy as np

import oracle
from synthetic import Intrinsics
from synthetic.configs import sequence_frame, small_orbit

K = Intrinsics(100.0, 100.0, 100.0, 100.0, 200, 200)
POSE = np.hstack([np.eye(3), np.zeros((3, 1))])
DIMS, VS, ORIGIN = (32, 32, 32), 0.01, (-0.16, -0.16, 0.84)


def plane_run(rule, weight_kind=oracle.WEIGHT_CONSTANT, w=1.0, w_max=math.inf, noise=oracle.NOISE_CONSTANT,
              coeff=0.2, n=12, seed=15, spread=0.003):
    vol = oracle.OracleVolume(DIMS, VS, ORIGIN, 4.0, 0.0, 4096)
    vol.set_rule(rule, weight_kind, w, w_max)
    rng = np.random.default_rng(seed)
    zs = []
    for o in rng.uniform(-spread, spread, n):
        z = np.float32(1.0 + o)
        zs.append(np.float64(z))
        vol.integrate(np.full((200, 200), z, np.float32), (K.fx, K.fy, K.cx, K.cy), POSE, noise, coeff)
    keys, T, P = vol.export()
    l = np.arange(8)
    lz = np.meshgrid(l, l, l, indexing="ij")[0].ravel()
    x = ORIGIN[2] + (keys[:, 2:3] * 8 + lz[None, :] + 0.5) * VS        # voxel centre z
    always = np.ones_like(x, bool)
    for z in zs:
        always &= np.abs(z - x) <= 0.04
    assert always.sum() > 1000
    m = np.stack([(z - x) / 0.04 for z in zs])                           # measurements per frame
    return T, P, m, always


def test_alg1_is_an_exponential_mean():
    w = 0.3
    T, P, m, ok = plane_run(oracle.RULE_RUNNING, w=w)
    n = m.shape[0]
    coef = np.array([(1 - w) ** (n - 1)] + [w * (1 - w) ** (n - k) for k in range(2, n + 1)])
    assert abs(coef.sum() - 1.0) < 1e-12
    expect = np.tensordot(coef, m, 1)
    np.testing.assert_allclose(T[ok], expect[ok], atol=1e-12)
    assert (P[ok] == 0.0).all()                                         # P is not used


def test_alg1_with_unit_weight_keeps_the_last_measurement():
    T, _, m, ok = plane_run(oracle.RULE_RUNNING, w=1.0)
    np.testing.assert_allclose(T[ok], m[-1][ok], atol=1e-15)


def test_alg2_without_cap_is_the_mean():
    T, W, m, ok = plane_run(oracle.RULE_WEIGHTED, w=0.7)
    np.testing.assert_allclose(T[ok], m.mean(0)[ok], atol=1e-12)
    np.testing.assert_allclose(W[ok], 0.7 * m.shape[0], rtol=1e-12)


def test_alg2_capped_at_one_weight_is_alg1_with_half():
    T2, W2, _, ok = plane_run(oracle.RULE_WEIGHTED, w=0.7, w_max=0.7)
    T1, _, _, _ = plane_run(oracle.RULE_RUNNING, w=0.5)
    np.testing.assert_allclose(T2[ok], T1[ok], atol=1e-12)
    assert (W2[ok] == 0.7).all()


def test_alg2_inverse_variance_equals_alg3_without_process_noise():
    # quadratic noise: p_k changes with the plane's depth from frame to frame
    T2, W2, _, ok = plane_run(oracle.RULE_WEIGHTED, oracle.WEIGHT_INV_VARIANCE, noise=oracle.NOISE_QUADRATIC,
                              coeff=0.0015, spread=0.02)
    T3, P3, _, ok3 = plane_run(oracle.RULE_KALMAN, noise=oracle.NOISE_QUADRATIC, coeff=0.0015, spread=0.02)
    assert (ok == ok3).all()
    live = np.abs(T3) <= 1
    assert (live == (np.abs(T2) <= 1)).all()
    np.testing.assert_allclose(T2[live], T3[live], atol=1e-12)
    np.testing.assert_allclose(W2[live] * P3[live], 1.0, rtol=1e-12)


def test_rules_allocate_the_same_blocks():
    spec = small_orbit(n_frames=3)
    out = []
    for rule, kw in ((oracle.RULE_KALMAN, {}), (oracle.RULE_RUNNING, dict(w=0.2)),
                     (oracle.RULE_WEIGHTED, dict(w=1.0, w_max=8.0))):
        vol = oracle.OracleVolume.from_grid(spec.grid)
        vol.set_rule(rule, **kw)
        for k in range(3):
            d, p = sequence_frame(spec, k)
            vol.integrate(d.numpy(), (spec.K.fx, spec.K.fy, spec.K.cx, spec.K.cy), p)
        keys, T, _ = oracle.sorted_blocks(*vol.export())
        out.append((keys, np.abs(T) <= 1))
    for keys, live in out[1:]:
        assert np.array_equal(keys, out[0][0])


def test_invalid_rules_rejected():
    vol = oracle.OracleVolume(DIMS, VS, ORIGIN)
    for args in ((3, 0, 1.0, 1.0), (oracle.RULE_RUNNING, 0, 1.5, 1.0), (oracle.RULE_RUNNING, 1, 0.5, 1.0),
                 (oracle.RULE_WEIGHTED, 0, 0.0, 1.0), (oracle.RULE_WEIGHTED, 0, 1.0, 0.0)):
        try:
            vol.set_rule(*args)
        except ValueError:
            continue
        raise AssertionError(args)

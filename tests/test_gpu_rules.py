"""Algorithms 1 and 2 as update rules of the HIP fusion against the oracle
(needs an MI355X).  Same bar as Algorithm 3: block sets exact, T within 1e-5
(delta units), P (the weight sum of Algorithm 2) within 1e-5 relative."""

import math

import numpy as np
import pytest
import torch

import oracle
from synthetic.configs import sequence_frame, small_orbit
from tests.parity import Kvec, compare_volumes, gpu_blocks, gpu_volume_for, oracle_volume_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tsdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd as m

    m.lib()
    return m


CASES = [
    ("running w=0.2", oracle.RULE_RUNNING, dict(w=0.2)),
    ("running w=1", oracle.RULE_RUNNING, dict(w=1.0)),
    ("weighted w=1 cap 8", oracle.RULE_WEIGHTED, dict(w=1.0, w_max=8.0)),
    ("weighted 1/p uncapped", oracle.RULE_WEIGHTED, dict(weight_kind=oracle.WEIGHT_INV_VARIANCE)),
]


@pytest.mark.parametrize("name,rule,kw", CASES, ids=[c[0] for c in CASES])
def test_rule_against_oracle(tsdf, name, rule, kw):
    spec = small_orbit(width=100, height=75, n_frames=6)   # ragged against the 16x16 preparation tiles
    gv = gpu_volume_for(spec)
    ov = oracle_volume_for(spec)
    gv.set_update_rule(rule, **kw)
    ov.set_rule(rule, **kw)
    for k in range(spec.n_frames):
        depth, pose = sequence_frame(spec, k)
        print(f"[rules] {name} frame {k}", flush=True)
        ost = ov.integrate(depth.numpy(), Kvec(spec.K), pose)
        gv.integrate(depth.cuda(), spec.K, pose)
        gst = gv.stats()
        assert gst["frame_updates"] == ost["updates"] and gst["frame_new_blocks"] == ost["new_blocks"]
    st = compare_volumes(gv, ov)
    print(f"[rules] {name}: {st}", flush=True)
    assert st["live"] > 10000


def test_weighted_inverse_variance_is_kalman_without_process_noise(tsdf):
    spec = small_orbit(width=100, height=75, n_frames=6)
    kal = gpu_volume_for(spec, q_hat=0.0)
    wgt = gpu_volume_for(spec, q_hat=0.0)
    wgt.set_update_rule(tsdf.RULE_WEIGHTED, tsdf.WEIGHT_INV_VARIANCE)
    for k in range(spec.n_frames):
        depth, pose = sequence_frame(spec, k)
        kal.integrate(depth.cuda(), spec.K, pose)
        wgt.integrate(depth.cuda(), spec.K, pose)
    kk, kT, kP = gpu_blocks(kal)
    wk, wT, wW = gpu_blocks(wgt)
    assert np.array_equal(kk, wk)
    live = np.abs(kT) <= 1
    assert (live == (np.abs(wT) <= 1)).all()
    assert np.abs(kT[live] - wT[live]).max() < 1e-5
    assert np.abs(kP[live] * wW[live] - 1.0).max() < 1e-5


def test_rule_validation(tsdf):
    spec = small_orbit(width=40, height=30, n_frames=1)
    v16 = gpu_volume_for(spec, storage=1)
    for args in ((3, 0, 1.0, 1.0), (1, 0, 0.0, 1.0), (1, 0, 1.5, 1.0), (1, 1, 0.5, 1.0), (2, 0, -1.0, 1.0),
                 (2, 0, 1.0, 0.0), (2, 2, 1.0, 1.0)):
        with pytest.raises(tsdf.TsdfError):
            v16.set_update_rule(*args)
    with pytest.raises(tsdf.TsdfError):
        v16.set_update_rule(2, 0, 1.0, math.inf)       # FP16 cannot hold an uncapped weight sum
    v16.set_update_rule(2, 0, 1.0, 65504.0)


@pytest.mark.parametrize("name,rule,kw", [("running fp16", oracle.RULE_RUNNING, dict(w=0.2)),
                                          ("weighted fp16", oracle.RULE_WEIGHTED, dict(w=1.0, w_max=8.0))])
def test_rule_fp16_against_oracle(tsdf, name, rule, kw):
    # FP16 storage rounds T and W on every store: same block set, T within
    # a few FP16 ulps of the oracle's (reported bound, not the FP32 gate)
    spec = small_orbit(width=100, height=75, n_frames=4)
    gv, ov = gpu_volume_for(spec, storage=1), oracle_volume_for(spec)
    gv.set_update_rule(rule, **kw)
    ov.set_rule(rule, **kw)
    for k in range(spec.n_frames):
        depth, pose = sequence_frame(spec, k)
        ov.integrate(depth.numpy(), Kvec(spec.K), pose)
        gv.integrate(depth.cuda(), spec.K, pose)
    st = compare_volumes(gv, ov, t_tol=4e-3, p_rtol=4e-3)
    print(f"[rules] {name}: {st}", flush=True)

"""tsdf_icp_run_noalloc (static scratch, no allocation) against tsdf_icp_run
with a caller workspace (needs an MI355X).

Two calls in a row on one device, the second on a smaller frame, so the
second runs over the scratch the first left behind: each must give the
records of tsdf_icp_run bit for bit, and its first iteration must match the
oracle to the bar of the ICP parity tests.
"""

import math

import numpy as np
import pytest
import torch

from oracle import icp as O
from synthetic import Intrinsics, look_at
from synthetic.configs import config_c2, sequence_frame
from synthetic.scenes import Scene, render_model_maps, sensor_depth

pytestmark = pytest.mark.gpu

CORNER = Scene(planes=np.array([[0.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, -0.8], [1.0, 0.0, 0.0, -0.7]]),
               spheres=np.array([[-0.3, 0.12, -0.4, 0.12]]))


@pytest.fixture(scope="module")
def tsdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd as m

    m.lib()
    return m


def orbit_case():
    spec = config_c2()
    K = spec.K
    model_pose = spec.poses[3]
    MV, MN = render_model_maps(spec.scene, K, model_pose, spec.near, spec.far)
    depth, _ = sequence_frame(spec, 4)
    params = O.IcpParams(dist_max=0.1, cos_min=math.cos(math.radians(30.0)), theta=0.005, shrink=True)
    return "640x480 orbit frame 4 against frame 3", K, depth, MV, MN, model_pose, params


def corner_case():
    K = Intrinsics(240.0, 240.0, 95.5, 71.5, 192, 144)
    true = look_at((0.3, 0.5, 0.4), (-0.3, 0.0, -0.4))
    depth = sensor_depth(CORNER, K, true, noise_seed=21)
    MV, MN = render_model_maps(CORNER, K, true)
    return "192x144 corner", K, depth, MV, MN, true, O.IcpParams(dist_max=0.05, cos_min=0.8)


def test_noalloc_equals_workspace_run_on_two_calls(tsdf):
    iters = 5
    for name, K, depth, MV, MN, model_pose, params in (orbit_case(), corner_case()):
        print(f"[no-alloc] {name}: {K.width}x{K.height}, {iters} iterations", flush=True)
        d, mv, mn = depth.cuda(), MV.cuda(), MN.cuda()
        ref = tsdf.Icp(K, params.dist_max, params.cos_min, params.theta, params.shrink, max_iters=iters)
        got = tsdf.Icp(K, params.dist_max, params.cos_min, params.theta, params.shrink, max_iters=iters)
        got.results.fill_(float("nan"))
        ref.run(d, mv, mn, model_pose, model_pose, iters)
        got.run_noalloc(d, mv, mn, model_pose, model_pose, iters)
        torch.cuda.synchronize()
        a = ref.results.cpu().numpy().view(np.uint64)
        b = got.results.cpu().numpy().view(np.uint64)
        assert np.array_equal(a, b), name
        g = got.result(0)
        o = O.icp_step(depth.numpy(), K.as_tuple(), MV.numpy(), MN.numpy(), model_pose, model_pose, params)
        assert g["N"] == o["N"] > 1000, name
        assert g["kept"] == o["kept"], name
        assert np.abs(g["pose"] - o["pose"]).max() <= 1e-10, name

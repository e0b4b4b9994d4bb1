"""ICP iteration of the HIP library against the oracle (needs an MI355X).

Inputs are synthetic: exact model maps of an analytic scene (as a raycast
lays them out) and noisy live depth maps from a nearby pose.  The pair count
must match exactly (every matching and rejection decision is taken in double
precision by both sides); the system, box, eigenvalues, increment and pose
must agree to the rounding of sums over the pairs.
"""

import math

import numpy as np
import pytest
import torch

from oracle import icp as O
from synthetic import Intrinsics, look_at
from synthetic.configs import config_c2, sequence_frame
from synthetic.scenes import Scene, render_depth, render_model_maps, sensor_depth

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


def perturbed(pose, r, t):
    out = pose.copy()
    out[:, :3] = O.rotation_increment(r) @ pose[:, :3]
    out[:, 3] += t
    return out


def compare(g, o, what):
    """GPU record g against oracle result o."""
    print(f"[icp] {what}: N {g['N']} / {o['N']}, kept {g['kept']} / {o['kept']}", flush=True)
    assert g["N"] == o["N"], what
    if o["N"] == 0:
        assert (g["pose"] == o["pose"]).all()
        return
    sc = np.abs(o["C"]).max()
    assert np.abs(g["C"] - o["C"]).max() <= 1e-9 * sc, what
    assert np.abs(g["b"] - o["b"]).max() <= 1e-9 * max(np.abs(o["b"]).max(), 1e-300) + 1e-300, what
    assert np.abs(g["m"] - o["m"]).max() <= 1e-15 and np.abs(g["S"] - o["S"]).max() <= 1e-15, what
    assert abs(g["residual2"] - o["residual2"]) <= 1e-9 * o["residual2"], what
    assert g["kept"] == o["kept"], what
    assert np.abs(g["lam"] - np.sort(o["lam"])).max() <= 1e-9 * np.abs(o["lam"]).max(), what
    assert np.abs(g["x"] - o["x"]).max() <= 1e-8 * max(np.abs(o["x"]).max(), 1e-6), what
    assert np.abs(g["pose"] - o["pose"]).max() <= 1e-10, what


def run_one(tsdf, depth, K, MV, MN, model_pose, pose, params):
    icp = tsdf.Icp(K, params.dist_max, params.cos_min, params.theta, params.shrink)
    icp.run(depth.cuda(), MV.cuda(), MN.cuda(), model_pose, pose, 1)
    torch.cuda.synchronize()
    g = icp.result(0)
    o = O.icp_step(depth.numpy(), K.as_tuple(), MV.numpy(), MN.numpy(), model_pose, pose, params)
    return g, o


@pytest.mark.parametrize("shrink,theta", [(True, 0.005), (False, 0.005), (True, -1.0), (False, -1.0)])
def test_one_iteration_small(tsdf, shrink, theta):
    K = Intrinsics(120.0, 120.0, 47.5, 35.5, 96, 72)   # ragged against 256-pixel workgroups
    model_pose = look_at((0.3, 0.5, 0.4), (-0.3, 0.0, -0.4))
    live_pose = perturbed(model_pose, [0.004, -0.006, 0.003], [0.005, -0.003, 0.004])
    depth = sensor_depth(CORNER, K, live_pose, noise_seed=11)
    MV, MN = render_model_maps(CORNER, K, model_pose)
    params = O.IcpParams(dist_max=0.05, cos_min=0.8, theta=theta, shrink=shrink)
    g, o = run_one(tsdf, depth, K, MV, MN, model_pose, model_pose, params)
    assert o["N"] > 3000
    compare(g, o, f"small shrink={shrink} theta={theta}")


def test_one_iteration_full_size_orbit(tsdf):
    # the 640x480 orbit sampled every 0.36 degrees: model maps of the scene
    # at frame 100, live depth of frame 101
    spec = config_c2(n_frames=1000)
    K = spec.K
    model_pose = spec.poses[100]
    MV, MN = render_model_maps(spec.scene, K, model_pose, spec.near, spec.far)
    depth, _ = sequence_frame(spec, 101)
    params = O.IcpParams(dist_max=0.02, cos_min=math.cos(math.radians(20.0)), theta=0.005, shrink=True)
    g, o = run_one(tsdf, depth, K, MV, MN, model_pose, model_pose, params)
    assert o["N"] > 30000
    compare(g, o, "orbit frame 101 against frame 100")


def test_chained_iterations_follow_the_oracle_and_converge(tsdf):
    K = Intrinsics(240.0, 240.0, 95.5, 71.5, 192, 144)
    true = look_at((0.3, 0.5, 0.4), (-0.3, 0.0, -0.4))
    depth = render_depth(CORNER, K, true).to(torch.float32)
    MV, MN = render_model_maps(CORNER, K, true)
    start = perturbed(true, [0.01, -0.015, 0.012], [0.008, -0.006, 0.01])
    params = O.IcpParams(dist_max=0.05, cos_min=0.8)
    icp = tsdf.Icp(K, params.dist_max, params.cos_min, params.theta, params.shrink)
    iters = 10
    icp.run(depth.cuda(), MV.cuda(), MN.cuda(), true, start, iters)
    torch.cuda.synchronize()
    est = start
    for k in range(iters):
        o = O.icp_step(depth.numpy(), K.as_tuple(), MV.numpy(), MN.numpy(), true, est, params)
        g = icp.result(k)
        assert g["N"] == o["N"], k
        assert np.abs(g["pose"] - o["pose"]).max() < 1e-9, k
        est = o["pose"]
    assert np.abs(g["pose"][:, 3] - true[:, 3]).max() < 1e-5
    assert np.abs(g["pose"][:, :3] - true[:, :3]).max() < 1e-5


def test_no_pairs_keeps_the_pose(tsdf):
    K = Intrinsics(120.0, 120.0, 47.5, 35.5, 96, 72)
    pose = look_at((0.3, 0.5, 0.4), (-0.3, 0.0, -0.4))
    depth = torch.zeros((K.height, K.width), dtype=torch.float32)
    MV, MN = render_model_maps(CORNER, K, pose)
    g, o = run_one(tsdf, depth, K, MV, MN, pose, pose, O.IcpParams())
    compare(g, o, "empty live map")
    assert g["N"] == 0


def test_registration_against_raycast_maps(tsdf):
    # end to end on the library's own model: fuse frames 0-9 of a finely
    # sampled orbit (0.36 degrees, 7.5 mm per frame), raycast at frame 9's
    # pose, register frame 10 starting from frame 9's pose; the estimate must
    # move most of the way to frame 10's true pose
    spec = config_c2(n_frames=1000)
    vol = tsdf.Volume.from_grid(spec.grid, max_width=spec.K.width, max_height=spec.K.height)
    for k in range(10):
        d, p = sequence_frame(spec, k)
        vol.integrate(d.cuda(), spec.K, p)
    vert, nrm = vol.raycast(spec.K, spec.poses[9])
    depth, truth = sequence_frame(spec, 10)
    icp = tsdf.Icp(spec.K, dist_max=0.05, cos_min=math.cos(math.radians(30.0)))
    icp.run(depth.cuda(), vert, nrm, spec.poses[9], spec.poses[9], 15)
    torch.cuda.synchronize()
    est = icp.result(14)["pose"]
    before = np.abs(spec.poses[9][:, 3] - truth[:, 3]).max()
    after = np.abs(est[:, 3] - truth[:, 3]).max()
    print(f"[icp] orbit frame 10: translation error {before:.4g} -> {after:.4g} m", flush=True)
    assert after < 0.1 * before


@pytest.mark.parametrize("w,h", [(1, 1), (2, 2), (17, 5), (257, 3)])
def test_tiny_and_ragged_frames(tsdf, w, h):
    # fewer pixels than one workgroup, a single row of workgroups, no pixel
    # with both neighbours (1x1): the pair count and pose still match
    K = Intrinsics(120.0 * max(w, h) / 96.0, 120.0 * max(w, h) / 96.0, (w - 1) / 2.0, (h - 1) / 2.0, w, h)
    model_pose = look_at((0.3, 0.5, 0.4), (-0.3, 0.0, -0.4))
    live_pose = perturbed(model_pose, [0.002, -0.001, 0.003], [0.002, 0.001, -0.002])
    depth = sensor_depth(CORNER, K, live_pose, noise_seed=5)
    MV, MN = render_model_maps(CORNER, K, model_pose)
    g, o = run_one(tsdf, depth, K, MV, MN, model_pose, model_pose, O.IcpParams(dist_max=0.05, cos_min=0.8))
    compare(g, o, f"{w}x{h}")


def test_tracking_loop_stays_on_the_true_trajectory(tsdf):
    # fuse, raycast and register on the system's own estimates (frame 0 at its
    # true pose) over 20 frames of the finely sampled orbit.  Directions the
    # threshold drops are not corrected, so the estimate drifts slowly; it
    # must stay far closer to the truth than the uncorrected trajectory (the
    # previous pose reused), which is off by the whole motion
    spec = config_c2(n_frames=1000)
    K = spec.K
    vol = tsdf.Volume.from_grid(spec.grid, max_width=K.width, max_height=K.height)
    icp = tsdf.Icp(K, dist_max=0.05, cos_min=math.cos(math.radians(30.0)))
    d0, est = sequence_frame(spec, 0)
    vol.integrate(d0.cuda(), K, est)
    worst = 0.0
    for k in range(1, 20):
        vert, nrm = vol.raycast(K, est)
        depth, truth = sequence_frame(spec, k)
        icp.run(depth.cuda(), vert, nrm, est, est, 10)
        torch.cuda.synchronize()
        est = icp.result(9)["pose"]
        vol.integrate(depth.cuda(), K, est)
        worst = max(worst, float(np.linalg.norm(est[:, 3] - truth[:, 3])))
    uncorrected = float(np.linalg.norm(spec.poses[0][:, 3] - spec.poses[19][:, 3]))
    print(f"[icp] tracking 20 frames: worst translation error {worst:.4g} m "
          f"(uncorrected {uncorrected:.4g} m)", flush=True)
    assert worst < 0.1 * uncorrected


def test_step_chain_equals_run_chain(tsdf):
    # tsdf_icp_step (cold eigen-decomposition every time, pose on the device)
    # and tsdf_icp_run (warm start from the previous eigenvectors) give the
    # same iterates to rounding
    K = Intrinsics(240.0, 240.0, 95.5, 71.5, 192, 144)
    true = look_at((0.3, 0.5, 0.4), (-0.3, 0.0, -0.4))
    depth = sensor_depth(CORNER, K, true, noise_seed=21).cuda()
    MV, MN = render_model_maps(CORNER, K, true)
    MV, MN = MV.cuda(), MN.cuda()
    start = perturbed(true, [0.01, -0.015, 0.012], [0.008, -0.006, 0.01])
    a = tsdf.Icp(K, 0.05, 0.8)
    b = tsdf.Icp(K, 0.05, 0.8)
    a.run(depth, MV, MN, true, start, 6)
    cur = torch.as_tensor(start.reshape(12)).cuda()
    for k in range(6):
        cur = b.step(depth, MV, MN, true, cur, k)
    torch.cuda.synchronize()
    for k in range(6):
        ra, rb = a.result(k), b.result(k)
        assert ra["N"] == rb["N"] and ra["kept"] == rb["kept"], k
        assert np.abs(ra["pose"] - rb["pose"]).max() < 1e-10, k
        assert np.abs(ra["lam"] - rb["lam"]).max() <= 1e-9 * np.abs(rb["lam"]).max(), k


def test_tracking_at_the_benchmark_frame_spacing(tsdf):
    # the benchmark's tracking leg on the first 20 frames of the 100-frame
    # orbit (7.5 cm and 3.6 degrees between frames): the estimate must stay
    # within the benchmark's drift bound on every frame
    import bench

    spec = config_c2()
    frames = [], []
    for k in range(20):
        d, p = sequence_frame(spec, k)
        frames[0].append(d.cuda())
        frames[1].append(p)
    rt = bench.run_tracking(spec, 20, frames, iters=10)
    print(f"[icp] tracking at the benchmark spacing: {rt}", flush=True)
    assert rt["frame_spacing_m"] > 0.07
    assert rt["tracking_ok"], rt

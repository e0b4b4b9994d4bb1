"""Argument errors at the C ABI on a live volume (needs an MI355X).

Every entry point checks its arguments on the host before it enqueues
anything: a bad pose (not a rotation, a reflection, non-finite), bad
intrinsics (NaN, a frame larger than the volume was sized for) or an unknown
noise model returns TSDF_EINVAL synchronously.  Afterwards the volume's frame
counter and statistics are unchanged, and output buffers keep the sentinel
written into them before the call.  The eviction call refuses a volume whose
device status is set even before the host has read that status back.
"""

import ctypes
import math

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def live():
    import paper_1311_7194_amd as tsdf
    from synthetic.configs import config_c1, sequence_frame

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    tsdf.lib()
    spec = config_c1()
    g = spec.grid
    print("[boundary] c1 volume, one frame fused", flush=True)
    vol = tsdf.Volume.from_grid(g, max_width=spec.K.width, max_height=spec.K.height)
    depth, pose = sequence_frame(spec, 0)
    depth = depth.cuda()
    vol.integrate(depth, spec.K, pose)
    torch.cuda.synchronize()
    return tsdf, spec, vol, depth, pose


def good_pose(pose):
    return np.ascontiguousarray(np.asarray(pose, np.float64).reshape(12))


def bad_poses(pose):
    p = np.asarray(pose, np.float64).reshape(3, 4)
    scaled = p.copy()
    scaled[:, :3] *= 1.01                                      # rows not unit length
    sheared = p.copy()
    sheared[0, 1] += 1e-3                                      # rows not orthogonal
    mirrored = p.copy()
    mirrored[:, 0] *= -1.0                                     # orthonormal, det = -1
    nan_t = p.copy()
    nan_t[1, 3] = math.nan
    inf_r = p.copy()
    inf_r[2, 2] = math.inf
    return {"scaled": scaled, "sheared": sheared, "mirrored": mirrored, "nan-translation": nan_t,
            "inf-rotation": inf_r}


def intrinsics(T, K, **kw):
    d = dict(fx=K.fx, fy=K.fy, cx=K.cx, cy=K.cy, width=K.width, height=K.height)
    d.update(kw)
    return T.Intrinsics(d["fx"], d["fy"], d["cx"], d["cy"], d["width"], d["height"])


def bad_intrinsics(T, K):
    return {"nan-fx": intrinsics(T, K, fx=math.nan), "inf-cy": intrinsics(T, K, cy=math.inf),
            "zero-fy": intrinsics(T, K, fy=0.0), "wider-than-volume": intrinsics(T, K, width=K.width + 8),
            "taller-than-volume": intrinsics(T, K, height=K.height + 1), "zero-width": intrinsics(T, K, width=0)}


def ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def call_integrate(tsdf, vol, depth, Kc, pose12, kind=0, coeff=0.0015):
    T = tsdf.tsdf
    noise = T.NoiseModel(kind, coeff, None)
    return T.lib().tsdf_integrate_frame(vol.handle, ptr(depth), ctypes.byref(Kc), pose12.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.byref(noise), None)


def call_raycast(tsdf, vol, Kc, pose12, vert, nrm):
    T = tsdf.tsdf
    return T.lib().tsdf_raycast(vol.handle, ctypes.byref(Kc), pose12.ctypes.data_as(ctypes.c_void_p), ptr(vert),
                                ptr(nrm), None)


def assert_untouched(tsdf, vol, before, sentinels):
    torch.cuda.synchronize()
    after = vol.stats()
    assert after == before, (before, after)
    for t in sentinels:
        assert bool((t == 7.0).all()), "an output buffer was written"


def test_integrate_rejects_bad_arguments(live):
    tsdf, spec, vol, depth, pose = live
    T = tsdf.tsdf
    K = spec.K
    before = vol.stats()
    Kc = intrinsics(T, K)
    for name, p in bad_poses(pose).items():
        rc = call_integrate(tsdf, vol, depth, Kc, good_pose(p))
        assert rc == T.EINVAL, (name, rc)
    for name, Kb in bad_intrinsics(T, K).items():
        rc = call_integrate(tsdf, vol, depth, Kb, good_pose(pose))
        assert rc == T.EINVAL, (name, rc)
    for kind, coeff in ((7, 0.0015), (-1, 0.0015), (0, math.nan), (0, -0.001), (2, 0.0015)):
        # kind 2 (learned) without network parameters is an error too
        rc = call_integrate(tsdf, vol, depth, Kc, good_pose(pose), kind, coeff)
        assert rc == T.EINVAL, (kind, coeff, rc)
    assert_untouched(tsdf, vol, before, [])
    assert before["frames"] == 1


def test_raycast_rejects_bad_arguments(live):
    tsdf, spec, vol, depth, pose = live
    T = tsdf.tsdf
    K = spec.K
    before = vol.stats()
    vert = torch.full((K.height + 1, K.width + 8, 4), 7.0, device="cuda")
    nrm = torch.full_like(vert, 7.0)
    Kc = intrinsics(T, K)
    for name, p in bad_poses(pose).items():
        assert call_raycast(tsdf, vol, Kc, good_pose(p), vert, nrm) == T.EINVAL, name
    for name, Kb in bad_intrinsics(T, K).items():
        assert call_raycast(tsdf, vol, Kb, good_pose(pose), vert, nrm) == T.EINVAL, name
    assert_untouched(tsdf, vol, before, [vert, nrm])


def test_icp_rejects_bad_arguments(live):
    tsdf, spec, vol, depth, pose = live
    T = tsdf.tsdf
    K = spec.K
    icp = tsdf.Icp(K, dist_max=0.05, cos_min=0.8, max_iters=2)
    vert, nrm = vol.raycast(K, pose)
    torch.cuda.synchronize()
    icp.results.fill_(7.0)
    L = T.lib()

    def run(Kc, model_pose, init_pose):
        return L.tsdf_icp_run(ptr(depth), ctypes.byref(Kc), ptr(vert), ptr(nrm),
                              model_pose.ctypes.data_as(ctypes.c_void_p), init_pose.ctypes.data_as(ctypes.c_void_p),
                              ctypes.byref(icp.params), 2, ptr(icp.workspace), ctypes.c_uint64(icp.workspace.numel()),
                              ptr(icp.results), None)

    Kc = intrinsics(T, K)
    for name, p in bad_poses(pose).items():
        assert run(Kc, good_pose(p), good_pose(pose)) == T.EINVAL, ("model", name)
        assert run(Kc, good_pose(pose), good_pose(p)) == T.EINVAL, ("initial", name)
    for name, Kb in bad_intrinsics(T, K).items():
        if name in ("wider-than-volume", "taller-than-volume"):
            continue   # ICP has no volume; its workspace is sized per frame below
        assert run(Kb, good_pose(pose), good_pose(pose)) == T.EINVAL, name
    # a frame larger than the workspace was sized for
    assert run(intrinsics(T, K, width=4 * K.width), good_pose(pose), good_pose(pose)) == T.EINVAL
    torch.cuda.synchronize()
    assert bool((icp.results == 7.0).all()), "a result record was written"


def test_evict_refuses_unread_overflow(live):
    """A pool overflow the host has not read back yet: eviction reads the
    device status itself and returns TSDF_EFULL without moving anything."""
    tsdf, spec, vol, depth, pose = live
    T = tsdf.tsdf
    g = spec.grid
    small = tsdf.Volume(g.dims, g.voxel_size, g.origin, g.trunc_voxels, 64, 128, max_width=spec.K.width,
                        max_height=spec.K.height, max_candidates=g.capacity_blocks)
    small.integrate(depth, spec.K, pose)    # needs ~500 blocks: the pool of 64 overflows
    work = torch.empty(int(T.lib().tsdf_evict_workspace_bytes(small.handle)), dtype=torch.uint8, device="cuda")
    keys = torch.full((64, 3), 7, dtype=torch.int32, device="cuda")
    Tb = torch.full((64, 512), 7.0, device="cuda")
    Pb = torch.full((64, 512), 7.0, device="cuda")
    lo = (ctypes.c_int32 * 3)(0, 0, 0)
    hi = (ctypes.c_int32 * 3)(3, 3, 3)
    n = ctypes.c_uint64(12345)
    rc = T.lib().tsdf_evict_blocks(small.handle, lo, hi, ptr(keys), ptr(Tb), ptr(Pb), ctypes.c_uint64(64), ptr(work),
                                   ctypes.c_uint64(work.numel()), ctypes.byref(n), None)
    assert rc == T.EFULL, rc
    assert n.value == 0
    torch.cuda.synchronize()
    assert bool((keys == 7).all()) and bool((Tb == 7.0).all()) and bool((Pb == 7.0).all())
    st = small.stats()
    assert st["status_flags"] & T.FLAG_POOL_FULL and st["allocated_blocks"] == 64

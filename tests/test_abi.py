"""The C ABI: every declared symbol is exported, host-side validation works.

These tests load libtsdf.so but make no call that reaches the GPU.
"""

import ctypes
import glob
import os
import re

import pytest

import paper_1311_7194_amd.tsdf as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(tsdf_[a-z0-9_]+)\s*\(", src, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(T.LIB_PATH):
        from paper_1311_7194_amd import build

        build.build()
    return T.lib()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "tsdf_integrate_frame" in names and "tsdf_raycast" in names
    for n in names:
        assert hasattr(lib, n), n


def desc(**kw):
    d = dict(dims=(256, 256, 256), voxel_size=0.004, origin=(-0.5, -0.5, 0.2), trunc_voxels=4.0,
             capacity_blocks=1 << 14, hash_slots=1 << 15, storage=0, q_hat=1e-4, max_width=640,
             max_height=480, max_candidates=0, dense_index=1)
    d.update(kw)
    return T.VolumeDesc((ctypes.c_int32 * 3)(*d["dims"]), d["voxel_size"], (ctypes.c_double * 3)(*d["origin"]),
                        d["trunc_voxels"], d["capacity_blocks"], d["hash_slots"], d["storage"], d["q_hat"],
                        d["max_width"], d["max_height"], d["max_candidates"], d["dense_index"])


def nbytes(lib, dd):
    out = ctypes.c_uint64(0)
    rc = lib.tsdf_volume_bytes(ctypes.byref(dd), ctypes.byref(out))
    return rc, out.value


def test_volume_bytes_accounts_for_pool_and_index(lib):
    rc, b32 = nbytes(lib, desc())
    assert rc == T.OK
    rc, b16 = nbytes(lib, desc(storage=1))
    assert rc == T.OK
    # pool: 2 arrays x (capacity + the chi block) x 512 voxels x element size
    assert b32 - b16 == 2 * ((1 << 14) + 1) * 512 * 2
    assert b32 >= 2 * (1 << 14) * 512 * 4 + 8 * (1 << 15)


@pytest.mark.parametrize("bad", [
    dict(dims=(250, 256, 256)),          # not a multiple of 8
    dict(dims=(16384, 8, 8)),            # beyond the 10-bit block key
    dict(voxel_size=0.0),
    dict(voxel_size=float("nan")),
    dict(trunc_voxels=-1.0),
    dict(capacity_blocks=0),
    dict(capacity_blocks=(1 << 22) + 1, hash_slots=1 << 24),   # beyond 32-bit pool offsets
    dict(hash_slots=3 << 14),            # not a power of two
    dict(hash_slots=1 << 14),            # below twice the capacity
    dict(storage=7),
    dict(q_hat=-1e-3),
    dict(max_width=0),
    dict(dense_index=2),
])
def test_invalid_descriptions_rejected(lib, bad):
    rc, _ = nbytes(lib, desc(**bad))
    assert rc == T.EINVAL


def test_null_arguments_rejected(lib):
    out = ctypes.c_uint64(0)
    assert lib.tsdf_volume_bytes(None, ctypes.byref(out)) == T.EINVAL
    assert lib.tsdf_create_volume(None, None, 0, None, None) == T.EINVAL
    h = ctypes.c_void_p()
    dd = desc()
    assert lib.tsdf_create_volume(ctypes.byref(dd), None, 1 << 30, None, ctypes.byref(h)) == T.EINVAL
    assert lib.tsdf_integrate_frame(None, None, None, None, None, None) == T.EINVAL
    assert lib.tsdf_raycast(None, None, None, None, None, None) == T.EINVAL
    assert lib.tsdf_query_stats(None, None) == T.EINVAL
    assert lib.tsdf_status_string(T.EFULL).decode().startswith("block pool")


def test_batch_host_validation(lib):
    assert lib.tsdf_batch_bytes(0) == 0
    assert lib.tsdf_batch_bytes(65) == 0
    assert lib.tsdf_batch_bytes(1) > 0 and lib.tsdf_batch_bytes(1) % 256 == 0
    assert lib.tsdf_batch_bytes(16) >= lib.tsdf_batch_bytes(1)
    h = ctypes.c_void_p()
    assert lib.tsdf_batch_create(None, None, 1, None, 0, ctypes.byref(h)) == T.EINVAL
    assert lib.tsdf_batch_create(None, None, 1, None, 0, None) == T.EINVAL
    assert lib.tsdf_batch_step(None, None, None, None, None, None, None) == T.EINVAL
    assert lib.tsdf_batch_set_graph(None, 1) == T.EINVAL
    assert lib.tsdf_batch_set_raycast_group(None, 4) == T.EINVAL
    assert lib.tsdf_batch_get_raycast_group(None) == 0
    lib.tsdf_batch_destroy(None)


def test_icp_host_validation(lib):
    assert lib.tsdf_icp_workspace_bytes(0, 480) == 0
    assert lib.tsdf_icp_workspace_bytes(640, 16385) == 0
    ws = lib.tsdf_icp_workspace_bytes(640, 480)
    assert ws == 512 * 40 * 8 + 36 * 8 and lib.tsdf_icp_workspace_bytes(16, 16) == 40 * 8 + 36 * 8
    assert ctypes.sizeof(T.IcpResult) == 600 and ctypes.sizeof(T.IcpParams) == 32
    K = T.Intrinsics(525.0, 525.0, 319.5, 239.5, 640, 480)
    pose = (ctypes.c_double * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails validation first

    def call(K=K, pose=pose, params=None, ws_bytes=ws, null=None):
        prm = params or T.IcpParams(0.02, 0.9, 0.005, 1, 0)
        args = [fake, ctypes.byref(K), fake, fake, pose, fake, ctypes.byref(prm), fake, ctypes.c_uint64(ws_bytes),
                fake, None]
        if null is not None:
            args[null] = None
        return lib.tsdf_icp_step(*args)

    for k in (0, 1, 2, 3, 4, 5, 6, 7, 9):
        assert call(null=k) == T.EINVAL, k
    assert call(ws_bytes=ws - 8) == T.EINVAL
    assert call(K=T.Intrinsics(0.0, 525.0, 319.5, 239.5, 640, 480)) == T.EINVAL
    assert call(K=T.Intrinsics(525.0, 525.0, 319.5, 239.5, 0, 480)) == T.EINVAL
    assert call(pose=(ctypes.c_double * 12)(2, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)) == T.EINVAL
    assert call(pose=(ctypes.c_double * 12)(-1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)) == T.EINVAL
    for bad in (T.IcpParams(0.0, 0.9, 0.005, 1, 0), T.IcpParams(float("nan"), 0.9, 0.005, 1, 0),
                T.IcpParams(0.02, 1.5, 0.005, 1, 0), T.IcpParams(0.02, 0.9, float("inf"), 1, 0),
                T.IcpParams(0.02, 0.9, 0.005, 2, 0)):
        assert call(params=bad) == T.EINVAL


def test_update_rule_validation_without_volume(lib):
    assert lib.tsdf_set_update_rule(None, 0, 0, 1.0, 1.0) == T.EINVAL


def test_icp_run_host_validation(lib):
    K = T.Intrinsics(525.0, 525.0, 319.5, 239.5, 640, 480)
    eye = (ctypes.c_double * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    bad = (ctypes.c_double * 12)(float("nan"), 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    prm = T.IcpParams(0.02, 0.9, 0.005, 1, 0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails validation first
    ws = ctypes.c_uint64(lib.tsdf_icp_workspace_bytes(640, 480))
    run = lambda pose, iters, res=fake: lib.tsdf_icp_run(fake, ctypes.byref(K), fake, fake, eye, pose,  # noqa: E731
                                                         ctypes.byref(prm), iters, fake, ws, res, None)
    assert run(eye, 0) == T.EINVAL and run(eye, 1025) == T.EINVAL
    assert run(bad, 1) == T.EINVAL and run(None, 1) == T.EINVAL and run(eye, 1, None) == T.EINVAL


def test_evict_host_validation_without_volume(lib):
    # a null volume is refused before anything touches a device
    assert lib.tsdf_evict_workspace_bytes(None) == 0
    lo = (ctypes.c_int32 * 3)(0, 0, 0)
    n = ctypes.c_uint64(7)
    work = ctypes.c_void_p(1 << 20)                     # never dereferenced: the call returns first
    assert lib.tsdf_evict_blocks(None, lo, lo, None, None, None, 0, work, 1 << 20, ctypes.byref(n), None) == T.EINVAL
    assert n.value == 7


def test_icp_run_noalloc_host_validation(lib):
    # every argument error is reported before the call looks up its device array
    K = T.Intrinsics(525.0, 525.0, 319.5, 239.5, 640, 480)
    eye = (ctypes.c_double * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    prm = T.IcpParams(0.02, 0.9, 0.005, 1, 0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails validation first

    def run(K=K, pose=eye, iters=1, null=None):
        args = [fake, ctypes.byref(K), fake, fake, eye, pose, ctypes.byref(prm), iters, fake, None]
        if null is not None:
            args[null] = None
        return lib.tsdf_icp_run_noalloc(*args)

    for k in (0, 1, 2, 3, 4, 5, 6, 8):
        assert run(null=k) == T.EINVAL, k
    assert run(iters=0) == T.EINVAL and run(iters=1025) == T.EINVAL
    assert run(K=T.Intrinsics(525.0, 525.0, 319.5, 239.5, 16385, 480)) == T.EINVAL
    assert run(K=T.Intrinsics(525.0, 525.0, 319.5, 239.5, 640, 0)) == T.EINVAL
    assert run(pose=(ctypes.c_double * 12)(-1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)) == T.EINVAL


def test_mesh_case_table_equals_the_oracle_table(lib):
    # the library derives its marching-cubes table at compile time, the
    # oracle at run time, each from the rule stated in tsdf_mesh.h; the two
    # derivations are separate code and must agree on every case
    import oracle

    oracle.build(force=False)
    edges = (ctypes.c_int32 * 15)()
    for c in range(256):
        n = lib.tsdf_mesh_case(c, edges)
        ref = oracle.mc_case(c)
        assert n == len(ref), c
        assert list(edges)[:3 * n] == ref.ravel().tolist(), c
        assert all(e == -1 for e in list(edges)[3 * n:]), c
    assert lib.tsdf_mesh_case(256, edges) == -1 and lib.tsdf_mesh_case(-1, edges) == -1
    assert lib.tsdf_mesh_case(0, None) == -1


def test_mesh_host_validation_without_volume(lib):
    assert lib.tsdf_mesh_workspace_bytes(None) == 0
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: the call returns first
    assert lib.tsdf_extract_mesh(None, fake, fake, None, 1, fake, 1 << 20, fake, None) == T.EINVAL


def test_batch_persistent_validation(lib):
    assert lib.tsdf_batch_set_persistent(None, 1) == T.EINVAL
    assert lib.tsdf_batch_set_persistent(None, 0) == T.EINVAL

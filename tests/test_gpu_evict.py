"""Block eviction of the HIP library against the oracle (needs an MI355X).

The evicted blocks and the kept volume must match the oracle's (block sets
exact, T within 1e-5, P within 1e-5 relative), fusion and raycast must go on
correctly after the rebuild, and streaming the evicted blocks back in must
give bitwise the volume that was never evicted."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
from synthetic.configs import sequence_frame, small_orbit
from tests.parity import (Kvec, compare_raycast, compare_volumes, gpu_blocks, gpu_volume_for,
                          oracle_volume_for)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tsdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd as m

    m.lib()
    return m


def box_of(keys):
    lo, hi = keys.min(0), keys.max(0)
    mid = (lo + hi) // 2
    return [int(lo[0]), int(lo[1]), int(lo[2])], [int(mid[0]), int(hi[1]), int(mid[2]) + 2]


def fuse(vol, spec, frames, gpu):
    for k in frames:
        d, p = sequence_frame(spec, k)
        if gpu:
            vol.integrate(d.cuda(), spec.K, p)
        else:
            vol.integrate(d.numpy(), Kvec(spec.K), p)


def test_evict_against_oracle(tsdf):
    spec = small_orbit(width=100, height=75, n_frames=6)
    gv, ov = gpu_volume_for(spec), oracle_volume_for(spec)
    fuse(gv, spec, range(3), True)
    fuse(ov, spec, range(3), False)
    lo, hi = box_of(ov.export()[0])
    gk, gT, gP = gv.evict(lo, hi)
    ok_, oT, oP = ov.evict(lo, hi)
    print(f"[evict] box {lo}..{hi}: gpu {len(gk)} / oracle {len(ok_)} evicted", flush=True)
    assert len(ok_) > 100
    a = oracle.sorted_blocks(gk.cpu().numpy(), gT.float().cpu().numpy().astype(np.float64),
                             gP.float().cpu().numpy().astype(np.float64))
    b = oracle.sorted_blocks(ok_, oT, oP)
    assert np.array_equal(a[0], b[0])
    live = np.abs(b[1]) <= 1
    assert np.array_equal(live, np.abs(a[1]) <= 1)
    assert np.abs(a[1][live] - b[1][live]).max() <= 1e-5
    assert (np.abs(a[2][live] - b[2][live]) <= 1e-5 * np.maximum(b[2][live], 1e-30)).all()
    assert gv.stats()["allocated_blocks"] == ov.n_blocks
    print("[evict] kept", compare_volumes(gv, ov), flush=True)
    # fusion and raycast after the rebuild
    fuse(gv, spec, range(3, 6), True)
    fuse(ov, spec, range(3, 6), False)
    print("[evict] after 3 more frames", compare_volumes(gv, ov), flush=True)
    pose = spec.poses[5]
    vert, nrm = gv.raycast(spec.K, pose)
    torch.cuda.synchronize()
    ovv, onn, ofl = ov.raycast(Kvec(spec.K), pose, spec.K.width, spec.K.height)
    rs = compare_raycast(vert.cpu().numpy(), nrm.cpu().numpy(), ovv, onn, ofl, pose, spec.grid.voxel_size)
    print("[evict] raycast", rs, flush=True)


@pytest.mark.parametrize("storage", [0, 1])
def test_stream_back_is_bitwise_lossless(tsdf, storage):
    spec = small_orbit(width=100, height=75, n_frames=5)
    ref, vol = gpu_volume_for(spec, storage=storage), gpu_volume_for(spec, storage=storage)
    fuse(ref, spec, range(5), True)
    fuse(vol, spec, range(3), True)
    lo, hi = box_of(vol.export()[0].cpu().numpy())
    k, T, P = vol.evict(lo, hi)
    assert len(k) > 0
    vol.import_blocks(k, T, P)
    fuse(vol, spec, range(3, 5), True)
    a, b = gpu_blocks(vol), gpu_blocks(ref)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_eviction_beyond_capacity_changes_nothing(tsdf):
    spec = small_orbit(width=100, height=75, n_frames=2)
    vol = gpu_volume_for(spec)
    fuse(vol, spec, range(2), True)
    before = gpu_blocks(vol)
    L = tsdf.lib()
    keys = torch.empty((1, 3), dtype=torch.int32, device="cuda")
    T = torch.empty((1, 512), device="cuda")
    work = torch.empty(int(L.tsdf_evict_workspace_bytes(vol.handle)), dtype=torch.uint8, device="cuda")
    n = ctypes.c_uint64(0)
    z = (ctypes.c_int32 * 3)(0, 0, 0)
    rc = L.tsdf_evict_blocks(vol.handle, z, z, ctypes.c_void_p(keys.data_ptr()), ctypes.c_void_p(T.data_ptr()),
                             ctypes.c_void_p(T.data_ptr()), ctypes.c_uint64(1), ctypes.c_void_p(work.data_ptr()),
                             ctypes.c_uint64(work.numel()), ctypes.byref(n), None)
    assert rc == tsdf.tsdf.ENOMEM and n.value == len(before[0])
    after = gpu_blocks(vol)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)


def test_evict_everything_then_fuse(tsdf):
    spec = small_orbit(width=100, height=75, n_frames=2)
    vol, fresh = gpu_volume_for(spec), gpu_volume_for(spec)
    fuse(vol, spec, [0], True)
    n0 = vol.stats()["allocated_blocks"]
    k, _, _ = vol.evict([1023, 1023, 1023], [1023, 1023, 1023])
    assert len(k) == n0 and vol.stats()["allocated_blocks"] == 0
    fuse(vol, spec, [1], True)
    fuse(fresh, spec, [1], True)
    a, b = gpu_blocks(vol), gpu_blocks(fresh)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_evict_edge_cases(tsdf):
    spec = small_orbit(width=100, height=75, n_frames=1)
    empty = gpu_volume_for(spec)
    k, _, _ = empty.evict([0, 0, 0], [0, 0, 0])
    assert len(k) == 0 and empty.stats()["allocated_blocks"] == 0
    vol = gpu_volume_for(spec)
    fuse(vol, spec, [0], True)
    before = gpu_blocks(vol)
    k, _, _ = vol.evict([0, 0, 0], [1023, 1023, 1023])          # the box holds every block
    assert len(k) == 0
    after = gpu_blocks(vol)
    for x, y in zip(before, after):
        assert np.array_equal(x, y)

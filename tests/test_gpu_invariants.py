"""Invariants of the HIP volume that hold whatever the schedule (needs an MI355X).

Blocks are allocated by racing workgroups, so pool order changes from run to
run; nothing else may.  Keys in the pool are unique and the pool is dense
(allocated_blocks live slots, no gaps), after fusion and after eviction, and
two runs of the same sequence in fresh volumes give bitwise the same sorted
volume and the same raycast maps, with and without the dense block index.
"""

import numpy as np
import pytest
import torch

from synthetic.configs import sequence_frame, small_orbit
from tests.parity import gpu_blocks, gpu_volume_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tsdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd as m

    m.lib()
    return m


def assert_pool_unique_and_dense(vol):
    keys, _, _ = vol.export()
    torch.cuda.synchronize()
    keys = keys.cpu().numpy()
    assert len(keys) == vol.stats()["allocated_blocks"]
    assert len(np.unique(keys, axis=0)) == len(keys)
    return len(keys)


@pytest.mark.parametrize("storage", [0, 1])
def test_repeated_runs_are_bitwise_identical(tsdf, storage):
    spec = small_orbit(width=100, height=75, n_frames=5)      # ragged against the 16x16 tiles
    runs = []
    for dense in (True, True, False):
        vol = gpu_volume_for(spec, storage=storage, dense_index=dense)
        for k in range(5):
            d, p = sequence_frame(spec, k)
            vol.integrate(d.cuda(), spec.K, p)
        print(f"[invariants] storage={storage} dense={dense}: {assert_pool_unique_and_dense(vol)} blocks",
              flush=True)
        maps = [vol.raycast(spec.K, spec.poses[k]) for k in (0, 4)]
        torch.cuda.synchronize()
        runs.append((gpu_blocks(vol), [(v.cpu(), n.cpu()) for v, n in maps]))
    (ref_blocks, ref_maps) = runs[0]
    assert int((ref_maps[0][0][..., 3] > 0).sum()) > 1000
    for blocks, maps in runs[1:]:
        for x, y in zip(blocks, ref_blocks):
            assert np.array_equal(x, y)
        for (v, n), (rv, rn) in zip(maps, ref_maps):
            assert torch.equal(v, rv) and torch.equal(n, rn)


def test_pool_stays_unique_and_dense_through_eviction(tsdf):
    spec = small_orbit(width=100, height=75, n_frames=6)
    vol = gpu_volume_for(spec)
    for k in range(3):
        d, p = sequence_frame(spec, k)
        vol.integrate(d.cuda(), spec.K, p)
    n0 = assert_pool_unique_and_dense(vol)
    keys = vol.export()[0].cpu().numpy()
    lo, hi = keys.min(0), keys.max(0)
    mid = (lo + hi) // 2
    k_out, _, _ = vol.evict([int(lo[0]), int(lo[1]), int(lo[2])], [int(mid[0]), int(hi[1]), int(hi[2])])
    n1 = assert_pool_unique_and_dense(vol)
    print(f"[invariants] eviction {n0} -> {n1} blocks ({len(k_out)} out)", flush=True)
    assert 0 < len(k_out) < n0 and n1 == n0 - len(k_out)
    kept = set(map(tuple, vol.export()[0].cpu().numpy()))
    assert not kept & set(map(tuple, k_out.cpu().numpy()))
    for k in range(3, 6):                                      # refill: new blocks land in the dense tail
        d, p = sequence_frame(spec, k)
        vol.integrate(d.cuda(), spec.K, p)
    assert assert_pool_unique_and_dense(vol) > n1

"""Pins of the oracle's block eviction (the volume shift that Section 8
names as future work): a partition of the store, and a lossless round trip
when the evicted blocks are streamed back in."""

import numpy as np

import oracle
from synthetic.configs import sequence_frame, small_orbit


def fused(spec, frames, vol=None):
    vol = vol or oracle.OracleVolume.from_grid(spec.grid)
    for k in frames:
        d, p = sequence_frame(spec, k)
        vol.integrate(d.numpy(), (spec.K.fx, spec.K.fy, spec.K.cx, spec.K.cy), p)
    return vol


def box_of(keys):
    lo, hi = keys.min(0), keys.max(0)
    mid = (lo + hi) // 2
    return np.array([lo[0], lo[1], lo[2]]), np.array([mid[0], hi[1], mid[2] + 2])


def test_eviction_partitions_the_store():
    spec = small_orbit(n_frames=3)
    vol = fused(spec, range(3))
    k0, T0, P0 = vol.export()
    lo, hi = box_of(k0)
    ke, Te, Pe = vol.evict(lo, hi)
    kk, Tk, Pk = vol.export()
    inside = lambda k: ((k >= lo) & (k <= hi)).all(1)   # noqa: E731
    assert len(ke) > 100 and len(kk) > 100 and len(ke) + len(kk) == len(k0)
    assert inside(kk).all() and not inside(ke).any()
    # both parts keep the original order and data
    pos = {tuple(k): i for i, k in enumerate(k0)}
    ik = np.array([pos[tuple(k)] for k in kk])
    ie = np.array([pos[tuple(k)] for k in ke])
    assert (np.diff(ik) > 0).all() and (np.diff(ie) > 0).all()
    assert np.array_equal(Tk, T0[ik]) and np.array_equal(Pk, P0[ik])
    assert np.array_equal(Te, T0[ie]) and np.array_equal(Pe, P0[ie])
    assert vol.n_blocks == len(kk)


def test_streaming_back_is_lossless():
    spec = small_orbit(n_frames=5)
    ref = fused(spec, range(5))
    vol = fused(spec, range(3))
    k0, _, _ = vol.export()
    lo, hi = box_of(k0)
    ke, Te, Pe = vol.evict(lo, hi)
    assert len(ke) > 0
    for key, t, p in zip(ke, Te, Pe):
        vol.set_block(key, t, p)
    fused(spec, range(3, 5), vol)
    a = oracle.sorted_blocks(*vol.export())
    b = oracle.sorted_blocks(*ref.export())
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_evicted_blocks_start_over():
    # a block evicted and seen again is allocated afresh: its first update
    # initialises it, as for a block never seen before
    spec = small_orbit(n_frames=2)
    vol = fused(spec, [0])
    k0, _, _ = vol.export()
    ke, _, _ = vol.evict(k0.max(0) + 1, k0.max(0) + 1)          # an empty box: evict everything
    assert len(ke) == len(k0) and vol.n_blocks == 0
    fused(spec, [1], vol)
    fresh = fused(spec, [1])
    a = oracle.sorted_blocks(*vol.export())
    b = oracle.sorted_blocks(*fresh.export())
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_eviction_larger_than_cap_changes_nothing():
    spec = small_orbit(n_frames=1)
    vol = fused(spec, [0])
    k0, T0, _ = vol.export()
    lib = oracle.lib()
    lo = np.zeros(3, np.int32)
    hi = np.zeros(3, np.int32)
    keys = np.zeros((4, 3), np.int32)
    T = np.zeros((4, 512))
    P = np.zeros((4, 512))
    n = lib.orc_evict(vol.h, oracle._ptr(lo), oracle._ptr(hi), oracle._ptr(keys), oracle._ptr(T), oracle._ptr(P), 4)
    assert n == -1 and vol.n_blocks == len(k0)
    k1, T1, _ = vol.export()
    assert np.array_equal(k0, k1) and np.array_equal(T0, T1)

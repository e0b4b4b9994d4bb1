"""CPU oracle for sparse TSDF fusion and raycasting — TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this package.  The HIP library never calls it and
shares no code with it.

The arithmetic lives in ``oracle.c`` (double precision, no FMA contraction);
this module compiles it with gcc and exposes it through ctypes with numpy
arrays.  ``mlp.py`` holds the oracle of the learned noise model.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = [os.path.join(_HERE, "oracle.c"), os.path.join(_HERE, "mlp.c"), os.path.join(_HERE, "mc.c")]

HIT, AMBIGUOUS, BISECT_INVALID, MARGINAL = 1, 2, 4, 8
NOISE_QUADRATIC, NOISE_CONSTANT, NOISE_PER_PIXEL = 0, 1, 2
RULE_KALMAN, RULE_RUNNING, RULE_WEIGHTED = 0, 1, 2       # Algorithms 3, 1 and 2
WEIGHT_CONSTANT, WEIGHT_INV_VARIANCE = 0, 1
CHI = 2.0


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain -O2, no contraction, OpenMP)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-Wall", "-o", tmp] + _SOURCES + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


class _Stats(ctypes.Structure):
    _fields_ = [("updates", ctypes.c_int64), ("new_blocks", ctypes.c_int64),
                ("ties", ctypes.c_int64), ("visited", ctypes.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [P, ctypes.c_double, P, ctypes.c_double, ctypes.c_double, ctypes.c_int64]
        L.orc_destroy.argtypes = [P]
        L.orc_block_count.restype = ctypes.c_int64
        L.orc_block_count.argtypes = [P]
        L.orc_integrate.restype = ctypes.c_int
        L.orc_integrate.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, P, P, ctypes.c_int32,
                                    ctypes.c_double, P, P]
        L.orc_raycast.restype = ctypes.c_int
        L.orc_raycast.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_int64, P, P, P,
                                  ctypes.c_int32]
        L.orc_sample.restype = ctypes.c_int
        L.orc_sample.argtypes = [P, P, P]
        L.orc_export.restype = ctypes.c_int64
        L.orc_export.argtypes = [P, P, P, P, ctypes.c_int64]
        L.orc_set_block.restype = ctypes.c_int
        L.orc_set_block.argtypes = [P, P, P, P]
        for name in ("orc_alg1_step",):
            getattr(L, name).argtypes = [P, ctypes.c_double, ctypes.c_double]
        L.orc_alg2_step.argtypes = [P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_set_rule.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        L.orc_set_threads.argtypes = [P, ctypes.c_int32]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_evict.argtypes = [P, P, P, P, P, P, ctypes.c_int64]
        L.orc_evict.restype = ctypes.c_int64
        L.orc_set_rule.restype = ctypes.c_int
        L.orc_mlp_param_count.restype = ctypes.c_int
        L.orc_bf16.restype = ctypes.c_double
        L.orc_bf16.argtypes = [ctypes.c_double]
        L.orc_mlp_features.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P]
        L.orc_mlp_forward.argtypes = [P, P, ctypes.c_int64, P]
        L.orc_mlp_loss_grad.restype = ctypes.c_double
        L.orc_mlp_loss_grad.argtypes = [P, P, P, ctypes.c_int64, P, ctypes.c_int32]
        L.orc_alg3_step.argtypes = [P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_mc_case.restype = ctypes.c_int
        L.orc_mc_case.argtypes = [ctypes.c_int32, P]
        L.orc_marching_cubes.restype = ctypes.c_int64
        L.orc_marching_cubes.argtypes = [P, P, P, P, ctypes.c_int64]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class OracleVolume:
    """Dense-offset-table sparse volume in double precision."""

    def __init__(self, dims: Sequence[int], voxel_size: float, origin: Sequence[float],
                 trunc_voxels: float = 4.0, q_hat: float = 1e-4, capacity_blocks: int = 1 << 16):
        self._dims = np.ascontiguousarray(np.asarray(dims, np.int32))
        o = _f64(origin)
        self.h = lib().orc_create(_ptr(self._dims), float(voxel_size), _ptr(o), float(trunc_voxels),
                                  float(q_hat), int(capacity_blocks))
        if not self.h:
            raise ValueError("oracle volume: invalid description")
        self.dims = tuple(int(x) for x in dims)
        self.voxel_size = float(voxel_size)
        self.origin = tuple(float(x) for x in origin)
        self.delta = float(trunc_voxels) * float(voxel_size)
        self.q_hat = float(q_hat)

    @classmethod
    def from_grid(cls, grid, q_hat: float = 1e-4, capacity_blocks: Optional[int] = None):
        return cls(grid.dims, grid.voxel_size, grid.origin, grid.trunc_voxels, q_hat,
                   capacity_blocks or grid.capacity_blocks)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    @property
    def n_blocks(self) -> int:
        return int(lib().orc_block_count(self.h))

    def set_rule(self, rule: int, weight_kind: int = WEIGHT_CONSTANT, w: float = 1.0, w_max: float = math.inf):
        """Update algorithm of later integrations (RULE_KALMAN, RULE_RUNNING, RULE_WEIGHTED)."""
        rc = lib().orc_set_rule(self.h, int(rule), int(weight_kind), float(w), float(w_max))
        if rc != 0:
            raise ValueError(f"oracle set_rule failed with status {rc}")

    def set_threads(self, n_threads: int):
        """Threads of later integrations (1: the serial loop over pixels)."""
        if lib().orc_set_threads(self.h, int(n_threads)) != 0:
            raise ValueError("oracle set_threads: n_threads must be >= 1")

    def integrate(self, depth, K, pose, noise_kind: int = NOISE_QUADRATIC, coeff: float = 0.0015,
                  phat: Optional[np.ndarray] = None) -> dict:
        d = np.ascontiguousarray(np.asarray(depth, np.float32))
        H, W = d.shape
        Kv = _f64(K[:4])
        pv = _f64(np.asarray(pose).reshape(12))
        ph = None if phat is None else _f64(phat).reshape(H * W)
        st = _Stats()
        rc = lib().orc_integrate(self.h, _ptr(d), W, H, _ptr(Kv), _ptr(pv), int(noise_kind),
                                 float(coeff), _ptr(ph), ctypes.byref(st))
        if rc != 0:
            raise RuntimeError(f"oracle integrate failed with status {rc}")
        return dict(updates=st.updates, new_blocks=st.new_blocks, ties=st.ties, visited=st.visited)

    def raycast(self, K, pose, width: int, height: int, pixels: Optional[np.ndarray] = None,
                n_threads: int = 1):
        """Returns vertex [n,4], normal [n,4] (float64) and flags [n] (int32)."""
        Kv = _f64(K[:4])
        pv = _f64(np.asarray(pose).reshape(12))
        if pixels is None:
            n = width * height
            px = None
        else:
            px = np.ascontiguousarray(np.asarray(pixels, np.int32).reshape(-1, 2))
            n = px.shape[0]
        vert = np.zeros((n, 4))
        nrm = np.zeros((n, 4))
        flags = np.zeros(n, np.int32)
        lib().orc_raycast(self.h, int(width), int(height), _ptr(Kv), _ptr(pv), _ptr(px), n, _ptr(vert),
                          _ptr(nrm), _ptr(flags), int(n_threads))
        return vert, nrm, flags

    def sample(self, p) -> Optional[float]:
        pv = _f64(p)
        F = np.zeros(1)
        ok = lib().orc_sample(self.h, _ptr(pv), _ptr(F))
        return float(F[0]) if ok else None

    def export(self):
        """keys [n,3] int32, T [n,512], P [n,512] in allocation order."""
        n = self.n_blocks
        keys = np.zeros((n, 3), np.int32)
        T = np.zeros((n, 512))
        P = np.zeros((n, 512))
        lib().orc_export(self.h, _ptr(keys), _ptr(T), _ptr(P), n)
        return keys, T, P

    def evict(self, lo, hi):
        """Remove the blocks outside the block box [lo, hi]; returns their keys [n,3], T, P [n,512]."""
        lo_, hi_ = np.ascontiguousarray(np.asarray(lo, np.int32)), np.ascontiguousarray(np.asarray(hi, np.int32))
        cap = self.n_blocks
        keys = np.zeros((max(cap, 1), 3), np.int32)
        T = np.zeros((max(cap, 1), 512))
        P = np.zeros((max(cap, 1), 512))
        n = lib().orc_evict(self.h, _ptr(lo_), _ptr(hi_), _ptr(keys), _ptr(T), _ptr(P), cap)
        if n < 0:
            raise RuntimeError("oracle evict failed")
        return keys[:n], T[:n], P[:n]

    def marching_cubes(self):
        """Triangles of the zero level set (mc.c): vertex ids [n,3] int64,
        edge parameters t [n,3] and world positions [n,3,3], float64."""
        n = int(lib().orc_marching_cubes(self.h, None, None, None, 0))
        vid = np.zeros((n, 3), np.int64)
        t = np.zeros((n, 3))
        pos = np.zeros((n, 3, 3))
        m = lib().orc_marching_cubes(self.h, _ptr(vid), _ptr(t), _ptr(pos), n)
        assert m == n
        return vid, t, pos

    def set_block(self, key, T, P=None):
        k = np.ascontiguousarray(np.asarray(key, np.int32))
        t = _f64(T).reshape(512)
        p = None if P is None else _f64(P).reshape(512)
        rc = lib().orc_set_block(self.h, _ptr(k), _ptr(t), _ptr(p))
        if rc != 0:
            raise RuntimeError(f"oracle set_block failed with status {rc}")


def alg1_step(T: float, Tk: float, w: float) -> float:
    t = np.array([T], np.float64)
    lib().orc_alg1_step(_ptr(t), float(Tk), float(w))
    return float(t[0])


def alg2_step(T: float, W: float, Tk: float, w: float, w_max: float):
    t = np.array([T], np.float64)
    ws = np.array([W], np.float64)
    lib().orc_alg2_step(_ptr(t), _ptr(ws), float(Tk), float(w), float(w_max))
    return float(t[0]), float(ws[0])


def alg3_step(T: float, P: float, Tk: float, pk: float, q: float):
    t = np.array([T], np.float64)
    p = np.array([P], np.float64)
    lib().orc_alg3_step(_ptr(t), _ptr(p), float(Tk), float(pk), float(q))
    return float(t[0]), float(p[0])


MLP_PARAMS = 1249


def bf16(x) -> np.ndarray:
    """bfloat16 round-to-nearest-even of float32(x), element-wise (via the oracle)."""
    a = np.asarray(x, np.float64)
    f = lib().orc_bf16
    return np.vectorize(f, otypes=[np.float64])(a) if a.ndim else np.float64(f(float(a)))


def mlp_features(depth, K):
    """Features [H*W, 4] and validity [H*W] of a depth map (see mlp.c)."""
    d = np.ascontiguousarray(np.asarray(depth, np.float32))
    H, W = d.shape
    feat = np.zeros((H * W, 4))
    valid = np.zeros(H * W, np.int32)
    lib().orc_mlp_features(_ptr(d), W, H, _ptr(_f64(K[:4])), _ptr(feat), _ptr(valid))
    return feat, valid.astype(bool)


def mlp_forward(params, x):
    p = _f64(params)
    xx = _f64(x).reshape(-1, 4)
    out = np.zeros(xx.shape[0])
    lib().orc_mlp_forward(_ptr(p), _ptr(xx), xx.shape[0], _ptr(out))
    return out


def mlp_loss_grad(params, x, r, round_bf16: bool = True):
    p = _f64(params)
    xx = _f64(x).reshape(-1, 4)
    rr = _f64(r).reshape(-1)
    g = np.zeros(MLP_PARAMS)
    loss = lib().orc_mlp_loss_grad(_ptr(p), _ptr(xx), _ptr(rr), xx.shape[0], _ptr(g), 1 if round_bf16 else 0)
    return float(loss), g


def mlp_variance(depth, K, params, delta: float, coeff: float = 0.0015) -> np.ndarray:
    """Per-pixel p_hat (delta^2 units) of the learned model: exp(s)/delta^2
    clamped to [p_q e^-4, p_q e^4] around the quadratic p_q, which also stands
    in where the features are undefined.  Flattened [H*W]."""
    d = np.asarray(depth, np.float32)
    feat, valid = mlp_features(d, K)
    s = mlp_forward(params, feat)
    D = d.reshape(-1).astype(np.float64)
    pq = (coeff * D * D / delta) ** 2
    pl = np.exp(s) / (delta * delta)
    return np.where(valid & (D > 0), np.clip(pl, pq * math.exp(-4.0), pq * math.exp(4.0)), pq)


MC_MAX_TRIS = 8


def mc_case(c: int) -> np.ndarray:
    """Triangles of marching-cubes case c as cube-edge numbers [n,3] (mc.c)."""
    e = np.zeros(3 * MC_MAX_TRIS, np.int32)
    n = lib().orc_mc_case(int(c), _ptr(e))
    if n < 0:
        raise ValueError("case index")
    return e[:3 * n].reshape(n, 3)


def sorted_blocks(keys: np.ndarray, *arrays):
    """Sort blocks by (z, y, x) key so two volumes can be compared."""
    order = np.lexsort((keys[:, 0], keys[:, 1], keys[:, 2]))
    return (keys[order],) + tuple(a[order] for a in arrays)

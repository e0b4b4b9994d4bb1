"""Oracle of one point-to-plane ICP iteration (Section 6) — TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of the
benchmark may import this module; the HIP library shares no code with it.

Plain FP64 numpy, following Section 6 step by step:

1. live points: every pixel with a valid depth is back-projected through its
   centre, ``x = (i - cx) / fx * D``, ``y = (j - cy) / fy * D``, ``z = D``;
   its normal is the cross product of the differences to its lower and right
   neighbours (lower x right, so it faces the camera), and exists only where
   both neighbours are valid;
2. both go to the world frame with the current pose estimate;
3. projective matching: the point is projected into the camera the model
   maps were rendered from and takes the model vertex q and normal n of the
   nearest pixel (same rounding as the fusion: ``floor(u + 1/2)``);
4. rejection by distance (``|p - q| <= dist_max``) and normal deviation (the
   angle between the live and the model normal at most ``acos(cos_min)``);
5. the 6x6 normal equations of the linearised functional
   ``sum ((R p + t - q) . n)^2`` with ``c = p x n`` (the Section 6 system);
6. optionally, the unit-cube scaling of the box that covers every matched p
   and q (centre m, diagonal S of its extents): ``c^ = S^-1 (c - m x n)``;
7. eigen-thresholding: the solution keeps only the eigen-directions of the
   system matrix whose eigenvalue divided by the number of pairs exceeds
   ``theta`` (0.005 in the paper);
8. back to the unscaled increment and on to the pose.

Readings (the paper leaves these open or states them inconsistently):

* the printed back-substitution ``r = S r^``, ``t = t^ + r x m`` does not
  invert the stated substitution: with ``c^ = S^-1 (c - m x n)`` the residual
  is ``(S r).c^ + (t + r x m).n + (p - q).n``, so ``r^ = S r`` and
  ``t^ = t + r x m``, i.e. ``r = S^-1 r^`` and ``t = t^ - r x m``; this is
  what is implemented (the scaled and unscaled solves then agree when no
  direction is dropped, which a test checks);
* the thresholded solution is ``sum_k v_k (v_k . b^) / lambda_k`` over the
  kept directions, equal to the paper's ``sum_k v_k (v_k . x^)`` whenever the
  system is invertible and still defined when it is not;
* a box extent of zero scales by 1;
* the rotation increment is ``Rz(gamma) Ry(beta) Rx(alpha)`` (rotations about
  x, then y, then z), whose first-order form is the paper's small-angle
  matrix; it is applied on the left: ``R' = R_inc R``, ``t' = R_inc t + t_inc``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np


@dataclass
class IcpParams:
    dist_max: float = 0.02        # metres
    cos_min: float = math.cos(math.radians(20.0))
    theta: float = 0.005          # eigenvalue threshold (per matched pair); < 0 keeps every direction
    shrink: bool = True           # solve the unit-cube-scaled system


def _cross(a, b):
    """a x b over the last axis, one component at a time (no reassociation)."""
    return np.stack([a[..., 1] * b[..., 2] - a[..., 2] * b[..., 1],
                     a[..., 2] * b[..., 0] - a[..., 0] * b[..., 2],
                     a[..., 0] * b[..., 1] - a[..., 1] * b[..., 0]], -1)


def _dot(a, b):
    return (a[..., 0] * b[..., 0] + a[..., 1] * b[..., 1]) + a[..., 2] * b[..., 2]


def _rotate(R, v):
    """R v for v [..., 3], each row as (R0 v0 + R1 v1) + R2 v2."""
    return np.stack([(R[a, 0] * v[..., 0] + R[a, 1] * v[..., 1]) + R[a, 2] * v[..., 2] for a in range(3)], -1)


def _rotate_t(R, v):
    """R^T v, component k as (R0k v0 + R1k v1) + R2k v2."""
    return np.stack([(R[0, k] * v[..., 0] + R[1, k] * v[..., 1]) + R[2, k] * v[..., 2] for k in range(3)], -1)


def live_points(depth, K):
    """Camera-frame points [H, W, 3], normals [H, W, 3] and their validity [H, W] (step 1)."""
    D = np.asarray(depth, np.float32).astype(np.float64)
    H, W = D.shape
    fx, fy, cx, cy = (float(k) for k in K[:4])
    valid = (D > 0) & np.isfinite(D)
    Dz = np.where(valid, D, 0.0)
    i = np.arange(W, dtype=np.float64)[None, :]
    j = np.arange(H, dtype=np.float64)[:, None]
    v = np.stack([(i - cx) / fx * Dz, (j - cy) / fy * Dz, Dz], -1)
    n = np.zeros_like(v)
    nvalid = np.zeros((H, W), bool)
    right = v[:-1, 1:] - v[:-1, :-1]
    down = v[1:, :-1] - v[:-1, :-1]
    n[:-1, :-1] = _cross(down, right)
    nvalid[:-1, :-1] = valid[:-1, :-1] & valid[:-1, 1:] & valid[1:, :-1]
    return v, n, valid & nvalid


def rotation_increment(r) -> np.ndarray:
    """Rz(gamma) Ry(beta) Rx(alpha) for r = (alpha, beta, gamma)."""
    a, b, g = (float(x) for x in r)
    Rx = np.array([[1, 0, 0], [0, math.cos(a), -math.sin(a)], [0, math.sin(a), math.cos(a)]])
    Ry = np.array([[math.cos(b), 0, math.sin(b)], [0, 1, 0], [-math.sin(b), 0, math.cos(b)]])
    Rz = np.array([[math.cos(g), -math.sin(g), 0], [math.sin(g), math.cos(g), 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def associate(depth, K, model_vertex, model_normal, model_pose, pose, params: IcpParams):
    """Steps 1-4: matched pairs (p, q, n) in world coordinates and, per live
    pixel, the index of the model pixel it matched (-1: no pair)."""
    K = [float(k) for k in K[:4]] + [int(K[4]), int(K[5])]
    fx, fy, cx, cy, W, H = K
    Rc, tc = np.asarray(pose, np.float64)[:, :3], np.asarray(pose, np.float64)[:, 3]
    Rm, tm = np.asarray(model_pose, np.float64)[:, :3], np.asarray(model_pose, np.float64)[:, 3]
    vc, nc, ok = live_points(depth, K)
    p = _rotate(Rc, vc) + tc
    nw = _rotate(Rc, nc)
    xm = _rotate_t(Rm, p - tm)
    zpos = xm[..., 2] > 0.0
    zs = np.where(zpos, xm[..., 2], 1.0)
    fu = np.floor(fx * xm[..., 0] / zs + cx + 0.5)
    fv = np.floor(fy * xm[..., 1] / zs + cy + 0.5)
    inside = zpos & (fu >= 0) & (fu < W) & (fv >= 0) & (fv < H)
    iu = np.where(inside, fu, 0).astype(np.int64)
    iv = np.where(inside, fv, 0).astype(np.int64)
    MV = np.asarray(model_vertex, np.float32).reshape(H, W, 4).astype(np.float64)
    MN = np.asarray(model_normal, np.float32).reshape(H, W, 4).astype(np.float64)
    q = MV[iv, iu, :3]
    n = MN[iv, iu, :3]
    has_model = MV[iv, iu, 3] > 0.0
    d = p - q
    near = _dot(d, d) <= params.dist_max * params.dist_max
    dot = _dot(nw, n)
    aligned = (dot > 0.0) & (dot * dot >= (params.cos_min * params.cos_min) * (_dot(nw, nw) * _dot(n, n)))
    m = ok & inside & has_model & near & aligned
    match = np.where(m, iv * W + iu, -1)
    return p[m], q[m], n[m], match


def normal_system(p, q, n, shrink: bool):
    """Steps 5-6: the 6x6 matrix C, right-hand side b and box (m, S)."""
    c = _cross(p, n)
    e = _dot(p - q, n)
    if shrink and len(p):
        pts = np.concatenate([p, q], 0)
        lo, hi = pts.min(0), pts.max(0)
        m = 0.5 * (lo + hi)
        S = hi - lo
        S = np.where(S > 0.0, S, 1.0)
        mn = _cross(np.broadcast_to(m, n.shape), n)
        c = (c - mn) / S
    else:
        m, S = np.zeros(3), np.ones(3)
    g = np.concatenate([c, n], 1)
    C = g.T @ g
    b = -(g.T @ e)
    return C, b, m, S, float(e @ e)


def thresholded_solve(C, b, N: int, theta: float):
    """Step 7: the solution restricted to eigen-directions with lambda/N > theta."""
    lam, V = np.linalg.eigh(C)
    keep = lam / max(N, 1) > theta if theta >= 0 else lam > 0.0
    keep &= lam > 0.0
    x = np.zeros(6)
    for k in np.nonzero(keep)[0]:
        x += V[:, k] * (V[:, k] @ b) / lam[k]
    return x, lam, keep


def icp_step(depth, K, model_vertex, model_normal, model_pose, pose, params: Optional[IcpParams] = None):
    """One iteration; returns the updated pose and everything the GPU reports."""
    params = params or IcpParams()
    pose = np.asarray(pose, np.float64).reshape(3, 4)
    p, q, n, match = associate(depth, K, model_vertex, model_normal, model_pose, pose, params)
    N = len(p)
    C, b, m, S, e2 = normal_system(p, q, n, params.shrink)
    out = dict(N=N, C=C, b=b, m=m, S=S, residual2=e2, match=match, pose=pose.copy(), x=np.zeros(6),
               lam=np.zeros(6), kept=0)
    if N == 0:
        return out
    xh, lam, keep = thresholded_solve(C, b, N, params.theta)
    r, t = xh[:3].copy(), xh[3:].copy()
    if params.shrink:
        r = r / S
        t = t - np.cross(r, m)
    Ri = rotation_increment(r)
    new = np.zeros((3, 4))
    new[:, :3] = Ri @ pose[:, :3]
    new[:, 3] = Ri @ pose[:, 3] + t
    out.update(x=np.concatenate([r, t]), lam=lam / N, kept=int(keep.sum()), pose=new)
    return out

"""Dense brute force over every voxel of a tiny grid, in numpy.

Evaluates the projective measurement of every voxel (not only those near a
depth sample) with the same double operations in the same order as the
method's definition, so its decisions are exactly the defined ones.  Used to
check that the oracle's sparse enumeration and allocation miss nothing.
"""

import numpy as np

CHI = 2.0


def dense_measure(dims, vs, origin, delta, depth, K, pose):
    """Returns (valid [Gz,Gy,Gx] bool, s [..] metres, i, j) for every voxel."""
    fx, fy, cx, cy = K
    H, W = depth.shape
    R = np.asarray(pose, np.float64)[:, :3]
    t = np.asarray(pose, np.float64)[:, 3]
    gx = np.arange(dims[0], dtype=np.float64)
    gy = np.arange(dims[1], dtype=np.float64)
    gz = np.arange(dims[2], dtype=np.float64)
    px = origin[0] + (gx + 0.5) * vs
    py = origin[1] + (gy + 0.5) * vs
    pz = origin[2] + (gz + 0.5) * vs
    dx = (px - t[0])[None, None, :]
    dy = (py - t[1])[None, :, None]
    dz = (pz - t[2])[:, None, None]
    xc = R[0, 0] * dx + R[1, 0] * dy + R[2, 0] * dz
    yc = R[0, 1] * dx + R[1, 1] * dy + R[2, 1] * dz
    zc = R[0, 2] * dx + R[1, 2] * dy + R[2, 2] * dz
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * xc / zc + cx
        v = fy * yc / zc + cy
    fu = np.floor(u + 0.5)
    fv = np.floor(v + 0.5)
    inside = (zc > 0) & (fu >= 0) & (fu < W) & (fv >= 0) & (fv < H)
    i = np.where(inside, fu, 0).astype(np.int64)
    j = np.where(inside, fv, 0).astype(np.int64)
    D = depth[j, i].astype(np.float64)
    ok = inside & (D > 0) & np.isfinite(D)
    s = D - zc
    valid = ok & (np.abs(s) <= delta)
    return valid, s, i, j


def dense_kalman(T, P, valid, Tk, pk, q):
    """Algorithm 3 on dense arrays (chi = |T| > 1)."""
    first = valid & (np.abs(T) > 1.0)
    upd = valid & ~first
    Pp = P + q
    K = Pp / (Pp + pk)
    Tn = T + K * (Tk - T)
    Pn = (1.0 - K) * Pp
    T = np.where(first, Tk, np.where(upd, Tn, T))
    P = np.where(first, pk, np.where(upd, Pn, P))
    T = np.where(valid & (np.abs(T) > 1.0), CHI, T)
    return T, P


def dense_to_blocks(T, P, alloc_mask):
    """Blocks [n,3] (x,y,z) of a dense allocation mask and their voxel data."""
    Gz, Gy, Gx = T.shape
    keys = np.argwhere(alloc_mask)[:, ::-1]  # (bx, by, bz)
    Tb = np.zeros((len(keys), 512))
    Pb = np.zeros((len(keys), 512))
    for n, (bx, by, bz) in enumerate(keys):
        Tb[n] = T[8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8].reshape(512)
        Pb[n] = P[8 * bz:8 * bz + 8, 8 * by:8 * by + 8, 8 * bx:8 * bx + 8].reshape(512)
    return keys.astype(np.int32), Tb, Pb


def block_mask(valid):
    Gz, Gy, Gx = valid.shape
    return valid.reshape(Gz // 8, 8, Gy // 8, 8, Gx // 8, 8).any(axis=(1, 3, 5))

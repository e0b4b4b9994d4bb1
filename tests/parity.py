"""Comparison helpers between the HIP library and the oracle (tests only)."""

import math

import numpy as np
import torch

import oracle

CHI = 2.0
T_TOL = 1e-5        # |T_hat_gpu - T_hat_oracle| in delta units
P_RTOL = 1e-5       # |P_hat_gpu - P_hat_oracle| / P_hat_oracle
Z_TOL_VOXELS = 1e-3 # raycast depth, in voxels
N_TOL_RAD = 1e-3    # normal angle


def Kvec(K):
    return (K.fx, K.fy, K.cx, K.cy)


FP16_U = 2.0 ** -11   # unit roundoff of FP16 (round to nearest)


def fp16_bounds(n):
    """Bounds on |dT_hat| and |dP_hat| / P_hat of FP16 storage after at most
    n updates of a voxel (one per frame), against exact arithmetic; the FP32
    form's own error (below 1e-5) is added by the caller.

    Each update reads the stored values, computes in FP32 and stores again.
    - P_hat: storing rounds by at most FP16_U relative.  Algorithm 3 maps a
      relative error e of P (P + Q keeps it) to (1 - K) e in K p_k, so the
      errors add up to at most n FP16_U (the first store included).
    - T_hat: T_hat lies in [-1, 1], where a store rounds by at most 2^-12
      absolutely.  T + K (T_k - T) takes an error of T as (1 - K) times
      itself, and an error e of P changes K by at most K (1 - K) e <= e / 4,
      which moves T by at most 2 e / 4 (|T_k - T| <= 2).  Update m therefore
      adds at most 2^-12 + m FP16_U / 2 = 2^-12 (1 + m), and n updates at most
      2^-12 (n + n (n + 1) / 2).
    """
    t = 2.0 ** -12 * (n + n * (n + 1) / 2.0)
    p = n * FP16_U
    return t, p


def gpu_blocks(vol):
    keys, T, P = vol.export()
    torch.cuda.synchronize()
    keys = keys.cpu().numpy()
    T = T.float().cpu().numpy().astype(np.float64)
    P = P.float().cpu().numpy().astype(np.float64)
    return oracle.sorted_blocks(keys, T, P)


def compare_volumes(gvol, ovol, t_tol=T_TOL, p_rtol=P_RTOL):
    """Block set bit-exact, live-voxel set exact, T and P within tolerance.

    Returns a dict of error statistics."""
    gk, gT, gP = gpu_blocks(gvol)
    ok_, oT, oP = oracle.sorted_blocks(*ovol.export())
    assert gk.shape == ok_.shape, f"block count differs: gpu {len(gk)} oracle {len(ok_)}"
    assert np.array_equal(gk, ok_), "block sets differ"
    glive = np.abs(gT) <= 1
    olive = np.abs(oT) <= 1
    chi_flips = int((glive != olive).sum())
    assert chi_flips <= 1e-6 * olive.size + 0, f"{chi_flips} voxels differ in chi status"
    both = glive & olive
    dT = np.abs(gT[both] - oT[both])
    rP = np.abs(gP[both] - oP[both]) / np.maximum(oP[both], 1e-30)
    stats = dict(blocks=len(gk), live=int(both.sum()), max_dT=float(dT.max(initial=0)),
                 max_rP=float(rP.max(initial=0)), chi_flips=chi_flips)
    assert stats["max_dT"] <= t_tol, stats
    assert stats["max_rP"] <= p_rtol, stats
    return stats


def camera_depth(vert, pose):
    R = np.asarray(pose)[:, :3]
    t = np.asarray(pose)[:, 3]
    return (vert[..., :3] - t) @ R[:, 2]


def compare_raycast(gv, gn, ov, on, oflags, pose, voxel, pixels=None):
    """gv, gn: gpu float4 maps (numpy [n,4]); ov, on, oflags: oracle per pixel."""
    gv = gv.reshape(-1, 4).astype(np.float64)
    gn = gn.reshape(-1, 4).astype(np.float64)
    if pixels is not None:
        gv = gv[pixels]
        gn = gn[pixels]
    ghit = gv[:, 3] > 0
    ohit = (oflags & oracle.HIT) > 0
    flagged = (oflags & (oracle.AMBIGUOUS | oracle.BISECT_INVALID | oracle.MARGINAL)) > 0
    mism = ghit != ohit
    unexplained = mism & ~flagged
    both = ghit & ohit & ~flagged
    dz = np.abs(camera_depth(gv[both], pose) - camera_depth(ov[both], pose)) / voxel
    cosang = np.clip((gn[both, :3] * on[both, :3]).sum(-1), -1, 1)
    ang = np.arccos(cosang)
    stats = dict(pixels=len(ohit), hits=int(ohit.sum()), gpu_hits=int(ghit.sum()), mismatched=int(mism.sum()),
                 unexplained=int(unexplained.sum()), max_dz_vox=float(dz.max(initial=0)),
                 max_normal_rad=float(ang.max(initial=0)), flagged=int(flagged.sum()))
    assert stats["unexplained"] <= max(1e-4 * len(ohit), 0), stats
    assert stats["max_dz_vox"] <= Z_TOL_VOXELS, stats
    assert stats["max_normal_rad"] <= N_TOL_RAD, stats
    return stats


def gpu_volume_for(spec, storage=0, q_hat=1e-4, capacity=None, max_wh=None, dense_index=True):
    from paper_1311_7194_amd import Volume

    g = spec.grid
    cap = capacity or g.capacity_blocks
    hs = 1
    while hs < 2 * cap:
        hs *= 2
    mw, mh = max_wh or (spec.K.width, spec.K.height)
    return Volume(g.dims, g.voxel_size, g.origin, g.trunc_voxels, cap, hs, storage, q_hat, mw, mh,
                  dense_index=dense_index)


def oracle_volume_for(spec, q_hat=1e-4, capacity=None):
    return oracle.OracleVolume.from_grid(spec.grid, q_hat=q_hat,
                                         capacity_blocks=capacity or spec.grid.capacity_blocks)

"""FP16 storage against the FP64 oracle and the FP32 form (needs an MI355X).

T_hat and P_hat stored in FP16 cannot meet the 1e-5 bound of the FP32 form
(one rounding is up to 2^-11 relative), so these checks use bounds derived
from that rounding (tests.parity.fp16_bounds, for one update per frame): the
block set and the chi status of every voxel must still be exact (neither
depends on stored values), |dT_hat| and |dP_hat| / P_hat within the derived
bounds plus the FP32 form's 1e-5, and the raycast depth within 0.1 voxel (a
T_hat error e moves the crossing by about e delta / cos(incidence), delta =
4 voxels; 0.1 voxel leaves room down to grazing incidence).
"""

import numpy as np
import pytest
import torch

from synthetic.configs import sequence_frame, small_orbit
from tests.parity import Kvec, camera_depth, fp16_bounds, gpu_blocks, gpu_volume_for, oracle_volume_for
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tsdf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd as m

    m.lib()
    return m


def stats(a, b, name):
    live = (np.abs(a[0]) <= 1) & (np.abs(b[0]) <= 1)
    dT = np.abs(a[0][live] - b[0][live])
    rP = np.abs(a[1][live] - b[1][live]) / np.maximum(b[1][live], 1e-30)
    out = dict(vs=name, live=int(live.sum()), max_dT=float(dT.max()), mean_dT=float(dT.mean()),
               rms_dT=float(np.sqrt((dT ** 2).mean())), max_rel_dP=float(rP.max()), mean_rel_dP=float(rP.mean()),
               chi_mismatch=int(((np.abs(a[0]) <= 1) != (np.abs(b[0]) <= 1)).sum()))
    print("[fp16]", out, flush=True)
    return out


def test_fp16_storage_error(tsdf):
    spec = small_orbit(width=100, height=75, n_frames=6, G=256, vs=0.008)
    g16 = gpu_volume_for(spec, storage=tsdf.F16)
    g32 = gpu_volume_for(spec, storage=tsdf.F32)
    ov = oracle_volume_for(spec)
    for k in range(spec.n_frames):
        d, p = sequence_frame(spec, k)
        ov.integrate(d.numpy(), Kvec(spec.K), p)
        g16.integrate(d.cuda(), spec.K, p)
        g32.integrate(d.cuda(), spec.K, p)
    k16, T16, P16 = gpu_blocks(g16)
    k32, T32, P32 = gpu_blocks(g32)
    ko, To, Po = oracle.sorted_blocks(*ov.export())
    assert np.array_equal(k16, ko) and np.array_equal(k32, ko)
    s64 = stats((T16, P16), (To, Po), "fp64-oracle")
    s32 = stats((T16, P16), (T32, P32), "fp32")
    t_bound, p_bound = fp16_bounds(spec.n_frames)
    print(f"[fp16] derived bounds after {spec.n_frames} updates: |dT| {t_bound:.3g}, |dP|/P {p_bound:.3g}", flush=True)
    for s in (s64, s32):
        assert s["chi_mismatch"] == 0
        assert s["max_dT"] <= t_bound + 1e-5
        assert s["max_rel_dP"] <= p_bound + 1e-5
    # raycast depth against the oracle's
    _, pose = sequence_frame(spec, 3)
    v16, n16 = g16.raycast(spec.K, pose)
    torch.cuda.synchronize()
    ovv, onn, ofl = ov.raycast(Kvec(spec.K), pose, spec.K.width, spec.K.height, n_threads=8)
    gv = v16.cpu().numpy().reshape(-1, 4).astype(np.float64)
    both = (gv[:, 3] > 0) & ((ofl & oracle.HIT) > 0) & ((ofl & (oracle.AMBIGUOUS | oracle.MARGINAL)) == 0)
    dz = np.abs(camera_depth(gv[both], pose) - camera_depth(ovv[both], pose)) / spec.grid.voxel_size
    print("[fp16] raycast vs oracle: pixels", int(both.sum()), "max dz (voxel)", float(dz.max()),
          "mean", float(dz.mean()), flush=True)
    assert both.sum() > 1000 and dz.max() <= 0.1

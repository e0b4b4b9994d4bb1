"""The learned noise model, trained on left-out residuals, against the
quadratic model on held-out sequences (needs an MI355X).

Reduced size: 4 training and 2 held-out orbit sequences of 24 frames at
320x240.  Gate: lower held-out negative log-likelihood on every held-out
sequence (the network describes the residual distribution better).

Fused-surface and TSDF errors are reported, not gated.  On these synthetic
inputs the quadratic model is the sensor model that generated the noise, so
a variance learned from residuals against a fused surface (which add that
surface's own error) cannot weight the measurements better: measured on 8
training and 4 held-out full-size orbits, the learned variance leaves the
surface 0.04 voxel further from the true surface on every held-out
sequence, whether the residuals are taken against a surface fused with or
without the frame.
"""

import pytest
import torch

pytestmark = pytest.mark.gpu


def test_learned_model_calibrates_heldout_residuals():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1311_7194_amd import learned_noise as LN

    res = LN.run(LN.small_size(), seed=0, log=lambda m: print(m, flush=True))
    print("[learned] nll diff", res["nll_diff"], "surface diff", res["surface_diff_vox"], "tsdf rms diff",
          res["tsdf_rms_diff_vox"], flush=True)
    assert res["residuals"] == "leave_out"
    assert res["final_loss"] < res["first_loss"]
    assert res["nll_diff"]["learned_better"] == res["nll_diff"]["n"]
    assert res["nll_diff"]["mean"] < 0.0

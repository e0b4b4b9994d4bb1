"""Learned noise model on the GPU against its oracle (needs an MI355X).

Gates: features (depth and radial exact to float rounding, edge distance
exact, incidence cosine within 1e-6); network output within 1e-4 relative on
99.9 % of samples (bfloat16 rounding of a hidden activation can flip where
the float and double pre-activations straddle a rounding boundary); batch
gradient within 1e-3 of its largest component; Adam equal to the oracle's
float64 update and to torch.optim.Adam.
"""

import math

import numpy as np
import pytest
import torch

import oracle
from synthetic.configs import config_c1, config_c2, sequence_frame, small_orbit
from tests.parity import Kvec, compare_volumes, gpu_volume_for, oracle_volume_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1311_7194_amd.mlp as M

    M.T.lib()
    return M


def trained_like_params(M, seed):
    """Random but realistic weights (bf16 values): init + a perturbation."""
    p = M.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p[M.OFF_W3:M.OFF_B3] += rng.normal(0, 0.3, 32)
    return oracle.bf16(p)


def frame_depth(n=0):
    spec = small_orbit(width=160, height=120, n_frames=2, G=256, vs=0.008)
    d, pose = sequence_frame(spec, n)
    return spec, d, pose


def test_features_match_oracle(mlp):
    spec, d, pose = frame_depth()
    feat, valid = mlp.features(d.cuda(), spec.K)
    torch.cuda.synchronize()
    of, ov = oracle.mlp_features(d.numpy(), Kvec(spec.K))
    g = feat.cpu().numpy().astype(np.float64)
    gv = valid.cpu().numpy().astype(bool)
    assert np.array_equal(gv, ov)
    print("[mlp] valid features", int(ov.sum()), "of", ov.size, flush=True)
    np.testing.assert_array_equal(g[:, 0], of[:, 0])
    np.testing.assert_allclose(g[:, 2], of[:, 2], atol=1e-7)
    np.testing.assert_allclose(g[:, 3], of[:, 3], rtol=1e-6)
    np.testing.assert_allclose(g[ov, 1], of[ov, 1], atol=1e-6)


@pytest.mark.parametrize("W,H", [(37, 29), (200, 5), (5, 70), (33, 17)])
def test_features_ragged_images_with_invalid_pixels(mlp, W, H):
    """Images smaller than or ragged against the 16x16 tiles, so that the
    48x48 feature window leaves the image on every side, with a depth step
    (discontinuities) and scattered invalid readings (0, negative, NaN,
    infinity) up to the borders."""
    from synthetic.scenes import Intrinsics

    rng = np.random.default_rng(1000 * W + H)
    jj, ii = np.mgrid[0:H, 0:W]
    d = (0.8 + 0.002 * ii + 0.003 * jj).astype(np.float32)
    d[:, W // 2:] += np.float32(0.1)
    bad = rng.random((H, W)) < 0.08
    d[bad] = np.array([0.0, -1.0, np.nan, np.inf], np.float32)[rng.integers(0, 4, int(bad.sum()))]
    K = Intrinsics(0.9 * W + 20.0, 0.9 * W + 20.0, W / 2.0 - 0.3, H / 2.0 + 0.2, W, H)
    feat, valid = mlp.features(torch.from_numpy(d).cuda(), K)
    torch.cuda.synchronize()
    of, ov = oracle.mlp_features(d, Kvec(K))
    g = feat.cpu().numpy().astype(np.float64)
    gv = valid.cpu().numpy().astype(bool)
    assert np.array_equal(gv, ov)
    print(f"[mlp] {W}x{H}: valid features {int(ov.sum())} of {ov.size}", flush=True)
    np.testing.assert_array_equal(g[:, 0], of[:, 0])
    np.testing.assert_allclose(g[:, 2], of[:, 2], atol=1e-7)
    np.testing.assert_allclose(g[:, 3], of[:, 3], rtol=1e-6)
    np.testing.assert_allclose(g[ov, 1], of[ov, 1], atol=1e-6)


def test_forward_matches_oracle(mlp):
    spec, d, pose = frame_depth()
    of, ov = oracle.mlp_features(d.numpy(), Kvec(spec.K))
    x = of[ov]
    p = trained_like_params(mlp, 1)
    s = mlp.forward(mlp.params_from_values(p), torch.tensor(x, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    got = s.cpu().numpy().astype(np.float64)
    ref = oracle.mlp_forward(p, x.astype(np.float32).astype(np.float64))
    rel = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    print("[mlp] forward n", len(ref), "max rel", rel.max(), "p99.9", np.quantile(rel, 0.999), flush=True)
    assert np.quantile(rel, 0.999) <= 1e-4
    assert rel.max() <= 2e-2


def test_loss_and_gradient_match_oracle(mlp):
    spec, d, pose = frame_depth()
    of, ov = oracle.mlp_features(d.numpy(), Kvec(spec.K))
    x = of[ov][:8192].astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(3)
    r = (0.0015 * x[:, 0] ** 2 * rng.normal(0, 1, len(x)) * (1 + 2 * (1 - x[:, 1]))).astype(np.float32)
    p = trained_like_params(mlp, 2)
    loss, grad = mlp.loss_grad(mlp.params_from_values(p), torch.tensor(x, dtype=torch.float32, device="cuda"),
                               torch.tensor(r, device="cuda"))
    torch.cuda.synchronize()
    oloss, og = oracle.mlp_loss_grad(p, x, r.astype(np.float64), round_bf16=True)
    g = grad.cpu().numpy().astype(np.float64)
    err = np.abs(g - og).max() / np.abs(og).max()
    print("[mlp] loss", loss.item(), oloss, "grad max err / max", err, flush=True)
    assert abs(loss.item() - oloss) <= 1e-4 * abs(oloss) + 1e-6
    assert err <= 1e-3


def test_batch_visiting_order(mlp):
    """A batch drawn through the affine visiting order equals the oracle on
    the permuted rows."""
    rng = np.random.default_rng(4)
    n = 1000
    x = np.column_stack([rng.uniform(0.3, 3, n), rng.uniform(0, 1, n), rng.uniform(0, 1, n),
                         rng.uniform(0, 0.7, n)]).astype(np.float32).astype(np.float64)
    r = rng.normal(0, 0.003, n).astype(np.float32)
    p = trained_like_params(mlp, 5)
    a, b, first, batch = 7, 13, 300, 250
    _, grad = mlp.loss_grad(mlp.params_from_values(p), torch.tensor(x, dtype=torch.float32, device="cuda"),
                            torch.tensor(r, device="cuda"), first=first, batch=batch, perm=(a, b))
    torch.cuda.synchronize()
    idx = (a * np.arange(first, first + batch) + b) % n
    _, og = oracle.mlp_loss_grad(p, x[idx], r[idx].astype(np.float64), round_bf16=True)
    assert np.abs(grad.cpu().numpy() - og).max() <= 1e-3 * np.abs(og).max()


def test_adam_matches_oracle_and_torch(mlp):
    """Five GPU Adam steps against the float64 oracle update (and against
    torch.optim.Adam); the bf16 parameters are the rounding of the masters."""
    from oracle.adam import adam_step

    p0 = trained_like_params(mlp, 6)
    tr = mlp.NoiseTrainer(p0, lr=1e-3)
    w = torch.nn.Parameter(torch.tensor(p0, dtype=torch.float32))
    opt = torch.optim.Adam([w], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    ow = np.asarray(p0, np.float32).astype(np.float64)
    om, ov = np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    rng = np.random.default_rng(7)
    for step in range(1, 6):
        g = rng.normal(0, 1e-2, mlp.N_PARAMS).astype(np.float32)
        tr.step(torch.tensor(g, device="cuda"))
        w.grad = torch.tensor(g)
        opt.step()
        ow, om, ov = adam_step(ow, om, ov, g.astype(np.float64), step)
    torch.cuda.synchronize()
    gpu = tr.master.cpu().numpy().astype(np.float64)
    # float32 state: each weight rounds at 2^-24 relative; 1 - 0.999^t in float
    # is off by 1.3e-5 relative, i.e. ~6e-9 per step of size ~lr
    np.testing.assert_allclose(gpu, ow, rtol=1e-6, atol=5e-8)
    np.testing.assert_allclose(tr.master.cpu().numpy(), w.detach().numpy(), rtol=1e-5, atol=1e-7)
    ref_bits = w.detach().to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(tr.params[:mlp.N_PARAMS].float().cpu().numpy(), ref_bits)


def test_integration_with_learned_variance(mlp):
    """MLP-mode integration against the oracle fed the oracle's own learned
    variance: identical block sets and update counts; values within the error
    that float features and network outputs carry (reported)."""
    spec = small_orbit(width=120, height=90, n_frames=3, G=256, vs=0.008)
    p = trained_like_params(mlp, 8)
    params = mlp.params_from_values(p)
    gv = gpu_volume_for(spec)
    ov = oracle_volume_for(spec)
    for k in range(3):
        d, pose = sequence_frame(spec, k)
        ph = oracle.mlp_variance(d.numpy(), Kvec(spec.K), p, spec.grid.delta)
        ost = ov.integrate(d.numpy(), Kvec(spec.K), pose, oracle.NOISE_PER_PIXEL, 0.0015, ph)
        gv.integrate(d.cuda(), spec.K, pose, 2, 0.0015, params)
        gst = gv.stats()
        assert gst["frame_updates"] == ost["updates"]
    st = compare_volumes(gv, ov, t_tol=1e-2, p_rtol=5e-2)
    print("[mlp] learned-variance integration", st, flush=True)


def test_integration_with_learned_variance_full_size(mlp):
    """The same check on the first two frames of the 640x480 orbit into the
    2048^3 grid, the configuration the benchmark's learned-noise line runs."""
    spec = config_c2(n_frames=2)
    p = trained_like_params(mlp, 8)
    params = mlp.params_from_values(p)
    gv = gpu_volume_for(spec)
    ov = oracle_volume_for(spec)
    for k in range(2):
        d, pose = sequence_frame(spec, k)
        ph = oracle.mlp_variance(d.numpy(), Kvec(spec.K), p, spec.grid.delta)
        ost = ov.integrate(d.numpy(), Kvec(spec.K), pose, oracle.NOISE_PER_PIXEL, 0.0015, ph)
        gv.integrate(d.cuda(), spec.K, pose, 2, 0.0015, params)
        gst = gv.stats()
        assert gst["frame_updates"] == ost["updates"] and gst["frame_new_blocks"] == ost["new_blocks"]
    st = compare_volumes(gv, ov, t_tol=1e-2, p_rtol=5e-2)
    print("[mlp] learned-variance integration, 640x480 orbit", st, flush=True)
    assert st["live"] > 1000000

"""Learned measurement-noise experiment: train on fused-surface residuals,
compare against the quadratic model on held-out sequences.

Training data: every sampled frame of a training sequence is compared with
a surface fused (with the quadratic noise model) from frames that exclude
it: the even frames are fused and the sampled odd frames raycast from their
own poses, then the other way round ("leave_out").  Each pixel with a
measurement, defined features and a hit gives (features, r = D - Z), the
residual of the measurement against that surface, so the residual holds the
sensor's noise and the fused surface's error but not the frame's own
contribution to that surface.  The older target ("fused": every frame fused,
then each sampled frame raycast against the surface it helped form) is kept
for comparison.  The network is trained on these with the Gaussian NLL (GPU
kernels, Adam).

Evaluation on held-out sequences, each fused twice (quadratic and learned):
  nll        mean NLL of the held-out residuals (of the quadratic-fused
             surface) under each model's predicted variance
  surface    mean |true SDF| at the raycast vertices, in voxels
  tsdf_rms   RMS of (T_hat * delta - true SDF) over stored voxels within the
             band, in voxels
reported per sequence and as paired differences (learned - quadratic).
"""

from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

import numpy as np
import torch

from . import mlp as M
from .tsdf import NOISE_MLP, NOISE_QUADRATIC, Volume

COEFF = 0.0015


@dataclasses.dataclass
class ExperimentSize:
    train_seeds: List[int]
    test_seeds: List[int]
    frames: int = 100
    sample_every: int = 5
    width: int = 640
    height: int = 480
    steps: int = 1500
    batch: int = 65536
    lr: float = 1e-3
    eval_every: int = 10
    residuals: str = "leave_out"   # or "fused"


def full_size() -> ExperimentSize:
    return ExperimentSize(list(range(100, 150)), list(range(200, 210)))


def small_size() -> ExperimentSize:
    return ExperimentSize([100, 101, 102, 103], [200, 201], frames=24, sample_every=3, width=320, height=240,
                          steps=300, batch=16384, eval_every=6)


def spec_for(seed: int, size: ExperimentSize):
    from synthetic.configs import config_c2

    s = config_c2(n_frames=size.frames, scene_seed=seed, width=size.width, height=size.height)
    # per-sequence noise and dropout seeds
    s.noise_seeds = [seed * 1000 + k for k in range(size.frames)]
    s.dropout_seeds = [seed * 1000 + 500 + k for k in range(size.frames)]
    return s


def _frames(spec):
    from synthetic.configs import sequence_frame

    out = []
    for k in range(spec.n_frames):
        d, p = sequence_frame(spec, k, device="cuda")
        out.append((d.contiguous(), p))
    return out


def _volume(spec):
    g = spec.grid
    return Volume(g.dims, g.voxel_size, g.origin, g.trunc_voxels, g.capacity_blocks, g.hash_slots,
                  max_width=spec.K.width, max_height=spec.K.height)


def fuse(vol: Volume, spec, frames, params: Optional[torch.Tensor] = None):
    vol.reset()
    for d, p in frames:
        if params is None:
            vol.integrate(d, spec.K, p, NOISE_QUADRATIC, COEFF)
        else:
            vol.integrate(d, spec.K, p, NOISE_MLP, COEFF, params)


def collect(vol: Volume, spec, frames, every: int, collector: M.SampleCollector):
    vert = torch.empty((spec.K.height, spec.K.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(vert)
    for k in range(0, len(frames), every):
        d, p = frames[k]
        vol.raycast(spec.K, p, vert, nrm)
        collector.add(d, spec.K, p, vert)


def collect_left_out(vol: Volume, spec, frames, every: int, collector: M.SampleCollector):
    """Residuals of every `every`-th frame against the surface fused from the
    frames of the other parity (the frame itself never contributes)."""
    vert = torch.empty((spec.K.height, spec.K.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(vert)
    for parity in (0, 1):
        fuse(vol, spec, [f for k, f in enumerate(frames) if k % 2 == parity])
        for k in range(0, len(frames), every):
            if k % 2 == parity:
                continue
            d, p = frames[k]
            vol.raycast(spec.K, p, vert, nrm)
            collector.add(d, spec.K, p, vert)


def residual_samples(vol: Volume, spec, frames, every: int, collector: M.SampleCollector, mode: str):
    if mode == "leave_out":
        collect_left_out(vol, spec, frames, every, collector)
    elif mode == "fused":
        fuse(vol, spec, frames)
        collect(vol, spec, frames, every, collector)
    else:
        raise ValueError(mode)


def quadratic_logvar(x: torch.Tensor) -> torch.Tensor:
    D = x[:, 0].double()
    return torch.log((COEFF * D * D) ** 2)


def nll(s: torch.Tensor, r: torch.Tensor) -> float:
    s = s.double()
    r = r.double()
    return float((0.5 * (s + r * r * torch.exp(-s))).mean())


def surface_error(vol: Volume, spec, frames, every: int) -> float:
    """Mean |true SDF| at raycast vertices (voxels)."""
    from synthetic import scene_sdf

    vert = torch.empty((spec.K.height, spec.K.width, 4), dtype=torch.float32, device="cuda")
    nrm = torch.empty_like(vert)
    tot, cnt = 0.0, 0
    for k in range(0, len(frames), every):
        d, p = frames[k]
        vol.raycast(spec.K, p, vert, nrm)
        v = vert.reshape(-1, 4)
        hit = v[:, 3] > 0
        x = v[hit, :3].double()
        sd = scene_sdf(spec.scene, x).abs() / spec.grid.voxel_size
        tot += float(sd.sum())
        cnt += int(hit.sum())
    return tot / max(cnt, 1)


def tsdf_rms(vol: Volume, spec) -> float:
    """RMS of stored distance minus true SDF over voxels in the band (voxels)."""
    from synthetic import scene_sdf

    keys, T, _ = vol.export()
    g = spec.grid
    l = torch.arange(8, device="cuda")
    lz, ly, lx = torch.meshgrid(l, l, l, indexing="ij")
    local = torch.stack([lx.reshape(-1), ly.reshape(-1), lz.reshape(-1)], -1)
    tot, cnt = 0.0, 0
    origin = torch.tensor(g.origin, dtype=torch.float64, device="cuda")
    for c0 in range(0, keys.shape[0], 4096):
        kb = keys[c0:c0 + 4096].long()
        gi = kb[:, None, :] * 8 + local[None]
        x = origin + (gi.double() + 0.5) * g.voxel_size
        t = T[c0:c0 + 4096].double()
        live = t.abs() <= 1
        sd = scene_sdf(spec.scene, x.reshape(-1, 3)).reshape(t.shape)
        band = live & (sd.abs() <= g.delta)
        err = (t * g.delta - sd)[band] / g.voxel_size
        tot += float((err * err).sum())
        cnt += int(band.sum())
    return math.sqrt(tot / max(cnt, 1))


def run(size: ExperimentSize, seed: int = 0, log=print) -> dict:
    t0 = time.time()
    spec0 = spec_for(size.train_seeds[0], size)
    vol = _volume(spec0)
    per_frame = size.width * size.height
    cap = len(size.train_seeds) * (size.frames // size.sample_every + 1) * per_frame
    collector = M.SampleCollector(cap, size.width, size.height)
    for s in size.train_seeds:
        spec = spec_for(s, size)
        frames = _frames(spec)
        residual_samples(vol, spec, frames, size.sample_every, collector, size.residuals)
        log(f"[learned] train seq {s}: {int(collector.count.item())} samples so far ({time.time() - t0:.0f} s)")
    x, r = collector.samples()
    trainer = M.NoiseTrainer(M.init_params(seed), lr=size.lr)
    t1 = time.time()
    losses = trainer.train(x, r, size.steps, size.batch, seed=seed)
    torch.cuda.synchronize()
    train_s = time.time() - t1
    log(f"[learned] trained {size.steps} steps on {x.shape[0]} samples in {train_s:.1f} s; "
        f"loss {losses[0]:.4f} -> {np.mean(losses[-20:]):.4f}")
    quad_train = nll(quadratic_logvar(x), r)
    rows = []
    for s in size.test_seeds:
        spec = spec_for(s, size)
        frames = _frames(spec)
        # held-out residuals of the training target's kind for the NLL, then
        # the quadratic fusion of the whole sequence for the surface metrics
        hc = M.SampleCollector(len(frames) // size.eval_every * per_frame + per_frame, size.width, size.height)
        residual_samples(vol, spec, frames, size.eval_every, hc, size.residuals)
        hx, hr = hc.samples()
        fuse(vol, spec, frames)
        nll_q = nll(quadratic_logvar(hx), hr)
        nll_l = nll(M.forward(trainer.params, hx), hr)
        surf_q = surface_error(vol, spec, frames, size.eval_every)
        rms_q = tsdf_rms(vol, spec)
        fuse(vol, spec, frames, trainer.params)
        surf_l = surface_error(vol, spec, frames, size.eval_every)
        rms_l = tsdf_rms(vol, spec)
        row = dict(seed=s, samples=int(hx.shape[0]), nll_quadratic=nll_q, nll_learned=nll_l,
                   surface_quadratic_vox=surf_q, surface_learned_vox=surf_l, tsdf_rms_quadratic_vox=rms_q,
                   tsdf_rms_learned_vox=rms_l)
        rows.append(row)
        log(f"[learned] held-out {s}: " + ", ".join(f"{k} {v:.5g}" if isinstance(v, float) else f"{k} {v}"
                                                     for k, v in row.items()))

    def paired(a, b):
        d = np.array([r[b] - r[a] for r in rows])
        return dict(mean=float(d.mean()), std=float(d.std(ddof=1)) if len(d) > 1 else 0.0,
                    learned_better=int((d < 0).sum()), n=len(d))

    return dict(residuals=size.residuals, train_samples=int(x.shape[0]), train_steps=size.steps,
                train_seconds=train_s,
                first_loss=losses[0], final_loss=float(np.mean(losses[-20:])), quadratic_train_nll=quad_train,
                heldout=rows, nll_diff=paired("nll_quadratic", "nll_learned"),
                surface_diff_vox=paired("surface_quadratic_vox", "surface_learned_vox"),
                tsdf_rms_diff_vox=paired("tsdf_rms_quadratic_vox", "tsdf_rms_learned_vox"),
                params=trainer.params, wall_s=time.time() - t0)


def main():
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser(description="learned measurement-noise experiment (one GPU)")
    ap.add_argument("--size", choices=["small", "full"], default="small")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--train", type=int, default=0, help="use only the first N training sequences (0: all)")
    ap.add_argument("--test", type=int, default=0, help="use only the first N held-out sequences (0: all)")
    ap.add_argument("--residuals", choices=["leave_out", "fused"], default="leave_out")
    a = ap.parse_args()
    size = full_size() if a.size == "full" else small_size()
    size.residuals = a.residuals
    if a.train:
        size.train_seeds = size.train_seeds[:a.train]
    if a.test:
        size.test_seeds = size.test_seeds[:a.test]
    res = run(size, a.seed, log=lambda m: print(m, file=sys.stderr, flush=True))
    res.pop("params")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

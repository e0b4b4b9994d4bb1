"""Binding and training driver of the learned measurement-noise model.

The network, its features, the loss gradient and the Adam step run in the
HIP kernels of libtsdf.so (``include/tsdf_mlp.h``); this module marshals
torch device tensors and loops over steps.
"""

from __future__ import annotations

import ctypes
import math
from typing import Optional

import numpy as np
import torch

from . import tsdf as T

N_PARAMS = 1249
N_PADDED = 1256
OFF_W1, OFF_B1, OFF_W2, OFF_B2, OFF_W3, OFF_B3 = 0, 128, 160, 1184, 1216, 1248

_bound = False


def _lib():
    global _bound
    L = T.lib()
    if not _bound:
        P = ctypes.c_void_p
        L.tsdf_mlp_features.argtypes = [P, P, P, P, P]
        L.tsdf_mlp_forward.argtypes = [P, P, ctypes.c_int64, P, P]
        L.tsdf_mlp_workspace_bytes.argtypes = [ctypes.c_int64]
        L.tsdf_mlp_workspace_bytes.restype = ctypes.c_uint64
        L.tsdf_mlp_loss_grad.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                         ctypes.c_uint64, P, P, P, P]
        L.tsdf_mlp_adam_step.argtypes = [P, P, P, P, P, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, P]
        L.tsdf_mlp_samples_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.tsdf_mlp_samples_workspace_bytes.restype = ctypes.c_uint64
        L.tsdf_mlp_collect_samples.argtypes = [P, P, P, P, P, P, P, P, ctypes.c_int64, P, P, P]
        for n in ("tsdf_mlp_features", "tsdf_mlp_forward", "tsdf_mlp_loss_grad", "tsdf_mlp_adam_step",
                  "tsdf_mlp_collect_samples"):
            getattr(L, n).restype = ctypes.c_int
        _bound = True
    return L


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def params_from_values(values, device="cuda") -> torch.Tensor:
    """bfloat16 parameter buffer (padded) from 1249 float values (rounded RNE)."""
    v = torch.zeros(N_PADDED, dtype=torch.float32)
    v[:N_PARAMS] = torch.as_tensor(np.asarray(values, np.float64)[:N_PARAMS], dtype=torch.float32)
    return v.to(torch.bfloat16).to(device)


def init_params(seed: int, coeff: float = 0.0015) -> np.ndarray:
    """Seeded initial weights (float64 values): small random layers and an
    output bias at the log-variance of the quadratic model at 1 m."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS)
    p[OFF_W1:OFF_B1] = rng.normal(0, 1.0 / math.sqrt(4), 128)
    p[OFF_W2:OFF_B2] = rng.normal(0, 1.0 / math.sqrt(32), 1024)
    p[OFF_W3:OFF_B3] = rng.normal(0, 0.1 / math.sqrt(32), 32)
    p[OFF_B3] = math.log(coeff * coeff)
    return p


def features(depth: torch.Tensor, K, stream=None):
    intr = T.make_intrinsics(K)
    H, W = depth.shape
    feat = torch.empty((H * W, 4), dtype=torch.float32, device=depth.device)
    valid = torch.empty(H * W, dtype=torch.uint8, device=depth.device)
    T._check(_lib().tsdf_mlp_features(_p(depth), ctypes.byref(intr), _p(feat), _p(valid), T.stream_handle(stream)),
             "tsdf_mlp_features")
    return feat, valid


def forward(params: torch.Tensor, x: torch.Tensor, stream=None) -> torch.Tensor:
    x = x.contiguous()
    s = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    T._check(_lib().tsdf_mlp_forward(_p(params), _p(x), x.shape[0], _p(s), T.stream_handle(stream)),
             "tsdf_mlp_forward")
    return s


def loss_grad(params: torch.Tensor, x: torch.Tensor, r: torch.Tensor, first: int = 0, batch: Optional[int] = None,
              perm=(1, 0), stream=None):
    n = x.shape[0]
    batch = n if batch is None else batch
    ws = torch.empty(int(_lib().tsdf_mlp_workspace_bytes(batch)) // 4 + 1, dtype=torch.float32, device=x.device)
    grad = torch.empty(N_PARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    T._check(_lib().tsdf_mlp_loss_grad(_p(params), _p(x), _p(r), n, first, batch, perm[0], perm[1], _p(ws), _p(grad),
                                       _p(loss), T.stream_handle(stream)), "tsdf_mlp_loss_grad")
    return loss, grad


def coprime_stride(n: int, rng: np.random.Generator) -> int:
    while True:
        a = int(rng.integers(1, max(n, 2)))
        if math.gcd(a, n) == 1:
            return a


class NoiseTrainer:
    """Adam on float32 master weights; the network used for inference is
    their bfloat16 rounding (``self.params``)."""

    def __init__(self, init_values: np.ndarray, lr=1e-3, betas=(0.9, 0.999), eps=1e-8, device="cuda"):
        self.master = torch.zeros(N_PARAMS, dtype=torch.float32, device=device)
        self.master.copy_(torch.as_tensor(np.asarray(init_values)[:N_PARAMS], dtype=torch.float32))
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.params = params_from_values(init_values, device)
        self.lr, self.betas, self.eps = lr, betas, eps
        self.step_count = 0

    def step(self, grad: torch.Tensor, stream=None):
        self.step_count += 1
        T._check(_lib().tsdf_mlp_adam_step(_p(self.master), _p(self.m), _p(self.v), _p(grad), _p(self.params),
                                           self.step_count, self.lr, self.betas[0], self.betas[1], self.eps,
                                           T.stream_handle(stream)), "tsdf_mlp_adam_step")

    def train(self, x: torch.Tensor, r: torch.Tensor, steps: int, batch: int = 65536, seed: int = 0,
              log_every: int = 0):
        """Mini-batch training over the samples (epochs visit them in a seeded
        affine order).  Returns the per-step mean losses (host list)."""
        n = x.shape[0]
        rng = np.random.default_rng(seed)
        ws = torch.empty(int(_lib().tsdf_mlp_workspace_bytes(batch)) // 4 + 1, dtype=torch.float32, device=x.device)
        grad = torch.empty(N_PARAMS, dtype=torch.float32, device=x.device)
        losses = torch.empty(steps, dtype=torch.float32, device=x.device)
        per_epoch = max(n // batch, 1)
        perm = (coprime_stride(n, rng), int(rng.integers(0, n)))
        for k in range(steps):
            e = k % per_epoch
            if e == 0 and k > 0:
                perm = (coprime_stride(n, rng), int(rng.integers(0, n)))
            b = min(batch, n)
            T._check(_lib().tsdf_mlp_loss_grad(_p(self.params), _p(x), _p(r), n, e * b, b, perm[0], perm[1], _p(ws),
                                               _p(grad), ctypes.c_void_p(losses.data_ptr() + 4 * k),
                                               T.stream_handle()), "tsdf_mlp_loss_grad")
            self.step(grad)
            if log_every and (k + 1) % log_every == 0:
                print(f"[mlp] step {k + 1}/{steps} loss {losses[k].item():.4f}", flush=True)
        return losses.cpu().tolist()


class SampleCollector:
    """Accumulates (features, residual) training rows from fused frames."""

    def __init__(self, capacity: int, max_w: int, max_h: int, device="cuda"):
        self.x = torch.empty((capacity, 4), dtype=torch.float32, device=device)
        self.r = torch.empty(capacity, dtype=torch.float32, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self.ws = torch.empty(int(_lib().tsdf_mlp_samples_workspace_bytes(max_w, max_h)) // 4 + 2,
                              dtype=torch.float32, device=device)
        self.capacity = capacity

    def add(self, depth: torch.Tensor, K, pose, vertex: torch.Tensor, stream=None):
        feat, valid = features(depth, K, stream)
        intr = T.make_intrinsics(K)
        p = T._pose_array(pose)
        T._check(_lib().tsdf_mlp_collect_samples(_p(depth), _p(feat), _p(valid), _p(vertex), ctypes.byref(intr),
                                                 p.ctypes.data_as(ctypes.c_void_p), _p(self.ws), _p(self.count),
                                                 self.capacity, _p(self.x), _p(self.r), T.stream_handle(stream)),
                 "tsdf_mlp_collect_samples")

    def samples(self):
        n = min(int(self.count.item()), self.capacity)
        return self.x[:n], self.r[:n]

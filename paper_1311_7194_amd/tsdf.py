"""ctypes binding of libtsdf over torch device tensors.

Argument marshalling only: every step of fusion and raycasting runs in the
HIP kernels of libtsdf.so.  torch provides device memory and streams.
The library must have been built (``paper_1311_7194_amd.build``); loading
fails loudly otherwise - there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsdf.so")

F32, F16 = 0, 1
NOISE_QUADRATIC, NOISE_CONSTANT, NOISE_MLP = 0, 1, 2
RULE_KALMAN, RULE_RUNNING, RULE_WEIGHTED = 0, 1, 2          # Algorithms 3, 1 and 2 (tsdf_update_rule)
WEIGHT_CONSTANT, WEIGHT_INV_VARIANCE = 0, 1
FLAG_POOL_FULL, FLAG_HASH_FULL, FLAG_CAND_FULL = 1, 2, 4
OK, EINVAL, ENOMEM, EFULL, EHIP, ESTATE = 0, 1, 2, 3, 4, 5

EXPORTED = [
    "tsdf_volume_bytes", "tsdf_create_volume", "tsdf_destroy_volume", "tsdf_reset_volume",
    "tsdf_integrate_frame", "tsdf_raycast", "tsdf_query_stats", "tsdf_export_blocks",
    "tsdf_import_blocks", "tsdf_status_string", "tsdf_set_timing", "tsdf_read_timing",
    "tsdf_set_raycast_group", "tsdf_get_raycast_group", "tsdf_autotune_raycast", "tsdf_raycast_footprint",
    "tsdf_batch_bytes", "tsdf_batch_create", "tsdf_batch_destroy", "tsdf_batch_set_graph",
    "tsdf_batch_set_raycast_group", "tsdf_batch_get_raycast_group", "tsdf_batch_step",
    "tsdf_batch_autotune_raycast", "tsdf_icp_workspace_bytes", "tsdf_icp_step", "tsdf_icp_run",
    "tsdf_set_update_rule", "tsdf_evict_workspace_bytes", "tsdf_evict_blocks", "tsdf_icp_run_noalloc",
    "tsdf_mesh_case", "tsdf_mesh_workspace_bytes", "tsdf_extract_mesh", "tsdf_batch_set_persistent",
    "tsdf_batch_set_fuse_grid", "tsdf_batch_get_fuse_grid", "tsdf_batch_autotune_fuse",
]


class VolumeDesc(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("voxel_size", ctypes.c_double),
                ("origin", ctypes.c_double * 3), ("trunc_voxels", ctypes.c_double),
                ("capacity_blocks", ctypes.c_uint32), ("hash_slots", ctypes.c_uint32),
                ("storage", ctypes.c_int32), ("q_hat", ctypes.c_double),
                ("max_width", ctypes.c_int32), ("max_height", ctypes.c_int32),
                ("max_candidates", ctypes.c_uint32), ("dense_index", ctypes.c_int32)]


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class NoiseModel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("coeff", ctypes.c_double), ("mlp_params_dev", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("allocated_blocks", ctypes.c_uint64), ("frame_candidates", ctypes.c_uint64),
                ("frame_new_blocks", ctypes.c_uint64), ("frame_updates", ctypes.c_uint64),
                ("frame_fresh_updates", ctypes.c_uint64), ("total_updates", ctypes.c_uint64),
                ("total_fresh_updates", ctypes.c_uint64), ("total_candidates", ctypes.c_uint64),
                ("total_new_blocks", ctypes.c_uint64), ("frames", ctypes.c_uint64),
                ("frame_touched_blocks", ctypes.c_uint64), ("total_touched_blocks", ctypes.c_uint64),
                ("status_flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "reserved"}


class Timing(ctypes.Structure):
    _fields_ = [("prep_ms", ctypes.c_double), ("fuse_ms", ctypes.c_double), ("range_ms", ctypes.c_double),
                ("raycast_ms", ctypes.c_double), ("prep_launches", ctypes.c_uint64),
                ("fuse_launches", ctypes.c_uint64), ("range_launches", ctypes.c_uint64),
                ("raycast_launches", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TsdfError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {lib().tsdf_status_string(status).decode()} (status {status})")
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1311_7194_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.tsdf_volume_bytes.argtypes = [P, P]
        L.tsdf_create_volume.argtypes = [P, P, ctypes.c_uint64, P, P]
        L.tsdf_destroy_volume.argtypes = [P]
        L.tsdf_destroy_volume.restype = None
        L.tsdf_reset_volume.argtypes = [P, P]
        L.tsdf_integrate_frame.argtypes = [P, P, P, P, P, P]
        L.tsdf_raycast.argtypes = [P, P, P, P, P, P]
        L.tsdf_raycast_footprint.argtypes = [P, P, P, P, P, P, P]
        L.tsdf_query_stats.argtypes = [P, P]
        L.tsdf_export_blocks.argtypes = [P, P, P, P, ctypes.c_uint64, P, P]
        L.tsdf_import_blocks.argtypes = [P, P, P, P, ctypes.c_uint64, P]
        L.tsdf_set_timing.argtypes = [P, ctypes.c_int32]
        L.tsdf_set_raycast_group.argtypes = [P, ctypes.c_int32]
        L.tsdf_evict_workspace_bytes.argtypes = [P]
        L.tsdf_evict_workspace_bytes.restype = ctypes.c_uint64
        L.tsdf_evict_blocks.argtypes = [P, P, P, P, P, P, ctypes.c_uint64, P, ctypes.c_uint64, P, P]
        L.tsdf_set_update_rule.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        L.tsdf_get_raycast_group.argtypes = [P]
        L.tsdf_autotune_raycast.argtypes = [P, P, P, P, P, ctypes.c_int32, P, P, P]
        L.tsdf_read_timing.argtypes = [P, P, ctypes.c_int32]
        L.tsdf_status_string.argtypes = [ctypes.c_int]
        L.tsdf_status_string.restype = ctypes.c_char_p
        L.tsdf_batch_bytes.argtypes = [ctypes.c_int32]
        L.tsdf_batch_bytes.restype = ctypes.c_uint64
        L.tsdf_batch_create.argtypes = [P, P, ctypes.c_int32, P, ctypes.c_uint64, P]
        L.tsdf_batch_destroy.argtypes = [P]
        L.tsdf_batch_destroy.restype = None
        L.tsdf_batch_set_graph.argtypes = [P, ctypes.c_int32]
        L.tsdf_batch_set_persistent.argtypes = [P, ctypes.c_int32]
        L.tsdf_batch_set_fuse_grid.argtypes = [P, ctypes.c_uint32]
        L.tsdf_batch_get_fuse_grid.argtypes = [P]
        L.tsdf_batch_get_fuse_grid.restype = ctypes.c_uint32
        L.tsdf_batch_autotune_fuse.argtypes = [P, P, P, P, P, P, ctypes.c_int32, P, P, P]
        L.tsdf_batch_set_raycast_group.argtypes = [P, ctypes.c_int32]
        L.tsdf_batch_get_raycast_group.argtypes = [P]
        L.tsdf_batch_step.argtypes = [P, P, P, P, P, P, P]
        L.tsdf_batch_autotune_raycast.argtypes = [P, P, P, P, ctypes.c_int32, P, P, P]
        L.tsdf_icp_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.tsdf_icp_workspace_bytes.restype = ctypes.c_uint64
        L.tsdf_icp_step.argtypes = [P, P, P, P, P, P, P, P, ctypes.c_uint64, P, P]
        L.tsdf_icp_run.argtypes = [P, P, P, P, P, P, P, ctypes.c_int32, P, ctypes.c_uint64, P, P]
        L.tsdf_icp_run_noalloc.argtypes = [P, P, P, P, P, P, P, ctypes.c_int32, P, P]
        L.tsdf_mesh_case.argtypes = [ctypes.c_int32, P]
        L.tsdf_mesh_workspace_bytes.argtypes = [P]
        L.tsdf_mesh_workspace_bytes.restype = ctypes.c_uint64
        L.tsdf_extract_mesh.argtypes = [P, P, P, P, ctypes.c_uint64, P, ctypes.c_uint64, P, P]
        for name in EXPORTED:
            if name not in ("tsdf_destroy_volume", "tsdf_status_string", "tsdf_batch_bytes", "tsdf_batch_destroy",
                            "tsdf_icp_workspace_bytes", "tsdf_evict_workspace_bytes", "tsdf_mesh_workspace_bytes",
                            "tsdf_batch_get_fuse_grid"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != OK:
        raise TsdfError(rc, what)


def stream_handle(stream: Optional[torch.cuda.Stream] = None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_intrinsics(K) -> Intrinsics:
    """From an object with fx, fy, cx, cy, width, height (or a 6-tuple)."""
    if hasattr(K, "fx"):
        return Intrinsics(K.fx, K.fy, K.cx, K.cy, K.width, K.height)
    fx, fy, cx, cy, w, h = K
    return Intrinsics(fx, fy, cx, cy, int(w), int(h))


def _pose_array(pose) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(pose, np.float64).reshape(12))
    return p


def _ptr(t: Optional[torch.Tensor]) -> Optional[ctypes.c_void_p]:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Volume:
    """A block-sparse TSDF volume living in one torch device buffer."""

    def __init__(self, dims: Sequence[int], voxel_size: float, origin: Sequence[float],
                 trunc_voxels: float = 4.0, capacity_blocks: int = 1 << 16, hash_slots: Optional[int] = None,
                 storage: int = F32, q_hat: float = 1e-4, max_width: int = 640, max_height: int = 480,
                 max_candidates: int = 0, dense_index: bool = True, device: str = "cuda",
                 stream: Optional[torch.cuda.Stream] = None):
        if hash_slots is None:
            hash_slots = 1
            while hash_slots < 2 * capacity_blocks:
                hash_slots *= 2
        self.desc = VolumeDesc((ctypes.c_int32 * 3)(*[int(d) for d in dims]), float(voxel_size),
                               (ctypes.c_double * 3)(*[float(o) for o in origin]), float(trunc_voxels),
                               int(capacity_blocks), int(hash_slots), int(storage), float(q_hat),
                               int(max_width), int(max_height), int(max_candidates), 1 if dense_index else 0)
        nbytes = ctypes.c_uint64(0)
        _check(lib().tsdf_volume_bytes(ctypes.byref(self.desc), ctypes.byref(nbytes)), "tsdf_volume_bytes")
        self.nbytes = int(nbytes.value)
        self.buffer = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.handle = ctypes.c_void_p()
        _check(lib().tsdf_create_volume(ctypes.byref(self.desc), _ptr(self.buffer), self.nbytes,
                                        stream_handle(stream), ctypes.byref(self.handle)),
               "tsdf_create_volume")
        self.storage = int(storage)
        self.dims = tuple(int(d) for d in dims)
        self.voxel_size = float(voxel_size)
        self.origin = tuple(float(o) for o in origin)
        self.delta = float(trunc_voxels) * float(voxel_size)
        self.capacity = int(capacity_blocks)

    @classmethod
    def from_grid(cls, grid, storage: int = F32, q_hat: float = 1e-4, max_width: int = 640,
                  max_height: int = 480, **kw):
        return cls(grid.dims, grid.voxel_size, grid.origin, grid.trunc_voxels, grid.capacity_blocks,
                   grid.hash_slots, storage, q_hat, max_width, max_height, **kw)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib().tsdf_destroy_volume(h)
            self.handle = None

    @property
    def elem_dtype(self):
        return torch.float16 if self.storage == F16 else torch.float32

    def reset(self, stream=None):
        _check(lib().tsdf_reset_volume(self.handle, stream_handle(stream)), "tsdf_reset_volume")

    def integrate(self, depth: torch.Tensor, K, pose, noise_kind: int = NOISE_QUADRATIC,
                  coeff: float = 0.0015, mlp_params: Optional[torch.Tensor] = None, stream=None):
        assert depth.is_cuda and depth.dtype == torch.float32 and depth.is_contiguous()
        intr = make_intrinsics(K)
        assert depth.shape == (intr.height, intr.width)
        p = _pose_array(pose)
        nm = NoiseModel(int(noise_kind), float(coeff),
                        ctypes.c_void_p(mlp_params.data_ptr()) if mlp_params is not None else None)
        _check(lib().tsdf_integrate_frame(self.handle, _ptr(depth), ctypes.byref(intr),
                                          p.ctypes.data_as(ctypes.c_void_p), ctypes.byref(nm),
                                          stream_handle(stream)), "tsdf_integrate_frame")

    def raycast(self, K, pose, vertex: Optional[torch.Tensor] = None, normal: Optional[torch.Tensor] = None,
                stream=None):
        intr = make_intrinsics(K)
        shape = (intr.height, intr.width, 4)
        if vertex is None:
            vertex = torch.empty(shape, dtype=torch.float32, device=self.buffer.device)
        if normal is None:
            normal = torch.empty(shape, dtype=torch.float32, device=self.buffer.device)
        assert vertex.shape == shape and normal.shape == shape
        assert vertex.is_contiguous() and normal.is_contiguous()
        p = _pose_array(pose)
        _check(lib().tsdf_raycast(self.handle, ctypes.byref(intr), p.ctypes.data_as(ctypes.c_void_p),
                                  _ptr(vertex), _ptr(normal), stream_handle(stream)), "tsdf_raycast")
        return vertex, normal

    def raycast_footprint(self, K, pose, vertex: Optional[torch.Tensor] = None,
                          normal: Optional[torch.Tensor] = None, stream=None):
        """(blocks read by the march, vertex, normal); synchronises."""
        intr = make_intrinsics(K)
        shape = (intr.height, intr.width, 4)
        if vertex is None:
            vertex = torch.empty(shape, dtype=torch.float32, device=self.buffer.device)
        if normal is None:
            normal = torch.empty(shape, dtype=torch.float32, device=self.buffer.device)
        assert vertex.shape == shape and normal.shape == shape
        p = _pose_array(pose)
        n = ctypes.c_uint64(0)
        _check(lib().tsdf_raycast_footprint(self.handle, ctypes.byref(intr), p.ctypes.data_as(ctypes.c_void_p),
                                            _ptr(vertex), _ptr(normal), ctypes.byref(n), stream_handle(stream)),
               "tsdf_raycast_footprint")
        return int(n.value), vertex, normal

    def stats(self) -> dict:
        st = Stats()
        _check(lib().tsdf_query_stats(self.handle, ctypes.byref(st)), "tsdf_query_stats")
        return st.as_dict()

    def set_update_rule(self, rule: int, weight_kind: int = WEIGHT_CONSTANT, w: float = 1.0,
                        w_max: float = math.inf):
        """Algorithm 3 (RULE_KALMAN, default), 1 (RULE_RUNNING) or 2 (RULE_WEIGHTED) for later integrations."""
        _check(lib().tsdf_set_update_rule(self.handle, int(rule), int(weight_kind), float(w), float(w_max)),
               "tsdf_set_update_rule")

    def set_raycast_group(self, group: int):
        _check(lib().tsdf_set_raycast_group(self.handle, int(group)), "tsdf_set_raycast_group")

    @property
    def raycast_group(self) -> int:
        return int(lib().tsdf_get_raycast_group(self.handle))

    def autotune_raycast(self, K, pose, reps: int = 3, stream=None):
        """Times every raycast group size on this view; keeps the fastest."""
        intr = make_intrinsics(K)
        vertex = torch.empty((intr.height, intr.width, 4), dtype=torch.float32, device=self.buffer.device)
        normal = torch.empty_like(vertex)
        p = _pose_array(pose)
        best = ctypes.c_int32(0)
        ms = ctypes.c_float(0)
        _check(lib().tsdf_autotune_raycast(self.handle, ctypes.byref(intr), p.ctypes.data_as(ctypes.c_void_p),
                                           _ptr(vertex), _ptr(normal), int(reps), stream_handle(stream),
                                           ctypes.byref(best), ctypes.byref(ms)), "tsdf_autotune_raycast")
        return int(best.value), float(ms.value)

    def set_timing(self, enable: bool):
        _check(lib().tsdf_set_timing(self.handle, 1 if enable else 0), "tsdf_set_timing")

    def read_timing(self, reset: bool = False) -> dict:
        t = Timing()
        _check(lib().tsdf_read_timing(self.handle, ctypes.byref(t), 1 if reset else 0), "tsdf_read_timing")
        return t.as_dict()

    def export(self, stream=None):
        """(keys [n,3] int32, T [n,512], P [n,512]) device tensors in pool order."""
        n = ctypes.c_uint64(0)
        _check(lib().tsdf_export_blocks(self.handle, None, None, None, 0, ctypes.byref(n),
                                        stream_handle(stream)), "tsdf_export_blocks")
        m = int(n.value)
        dev = self.buffer.device
        keys = torch.empty((max(m, 1), 3), dtype=torch.int32, device=dev)
        T = torch.empty((max(m, 1), 512), dtype=self.elem_dtype, device=dev)
        P = torch.empty((max(m, 1), 512), dtype=self.elem_dtype, device=dev)
        if m:
            _check(lib().tsdf_export_blocks(self.handle, _ptr(keys), _ptr(T), _ptr(P), m, ctypes.byref(n),
                                            stream_handle(stream)), "tsdf_export_blocks")
        return keys[:m], T[:m], P[:m]

    def evict(self, lo, hi, stream=None):
        """Remove the blocks outside the block-coordinate box [lo, hi] and
        return them as (keys [n,3] int32, T, P [n,512]) device tensors."""
        cap = max(int(self.stats()["allocated_blocks"]), 1)
        dev = self.buffer.device
        keys = torch.empty((cap, 3), dtype=torch.int32, device=dev)
        T = torch.empty((cap, 512), dtype=self.elem_dtype, device=dev)
        P = torch.empty_like(T)
        work = torch.empty(int(lib().tsdf_evict_workspace_bytes(self.handle)), dtype=torch.uint8, device=dev)
        lo_ = (ctypes.c_int32 * 3)(*[int(x) for x in lo])
        hi_ = (ctypes.c_int32 * 3)(*[int(x) for x in hi])
        n = ctypes.c_uint64(0)
        _check(lib().tsdf_evict_blocks(self.handle, lo_, hi_, _ptr(keys), _ptr(T), _ptr(P), ctypes.c_uint64(cap),
                                       _ptr(work), ctypes.c_uint64(work.numel()), ctypes.byref(n),
                                       stream_handle(stream)), "tsdf_evict_blocks")
        m = int(n.value)
        return keys[:m], T[:m], P[:m]

    def mesh_workspace(self) -> torch.Tensor:
        """A device workspace for extract_mesh (reusable across calls)."""
        return torch.empty(int(lib().tsdf_mesh_workspace_bytes(self.handle)), dtype=torch.uint8,
                           device=self.buffer.device)

    def extract_mesh_into(self, vid: Optional[torch.Tensor], t: Optional[torch.Tensor], xyz: Optional[torch.Tensor],
                          count: torch.Tensor, work: torch.Tensor, stream=None):
        """tsdf_extract_mesh into caller tensors (no synchronisation): vid
        int64 [cap,3], t float32 [cap,3], xyz float32 [cap,3,3] or None,
        count a one-element int64 device tensor."""
        cap = 0 if vid is None else int(vid.shape[0])
        _check(lib().tsdf_extract_mesh(self.handle, _ptr(vid), _ptr(t), _ptr(xyz), ctypes.c_uint64(cap),
                                       _ptr(work), ctypes.c_uint64(work.numel()), _ptr(count),
                                       stream_handle(stream)), "tsdf_extract_mesh")

    def extract_mesh(self, with_xyz: bool = True, stream=None):
        """Marching cubes over the allocated blocks (tsdf_mesh.h): returns
        (vertex ids [n,3] int64, t [n,3] float32, world positions [n,3,3]
        float32 or None) as device tensors.  Counts first, then extracts."""
        dev = self.buffer.device
        work = self.mesh_workspace()
        count = torch.zeros(1, dtype=torch.int64, device=dev)
        self.extract_mesh_into(None, None, None, count, work, stream)
        n = int(count.item())
        vid = torch.empty((max(n, 1), 3), dtype=torch.int64, device=dev)
        t = torch.empty((max(n, 1), 3), dtype=torch.float32, device=dev)
        xyz = torch.empty((max(n, 1), 3, 3), dtype=torch.float32, device=dev) if with_xyz else None
        self.extract_mesh_into(vid, t, xyz, count, work, stream)
        return vid[:n], t[:n], (xyz[:n] if with_xyz else None)

    def import_blocks(self, keys: torch.Tensor, T: torch.Tensor, P: torch.Tensor, stream=None):
        keys = keys.to(device=self.buffer.device, dtype=torch.int32).contiguous()
        T = T.to(device=self.buffer.device, dtype=self.elem_dtype).contiguous()
        P = P.to(device=self.buffer.device, dtype=self.elem_dtype).contiguous()
        n = keys.shape[0]
        _check(lib().tsdf_import_blocks(self.handle, _ptr(keys), _ptr(T), _ptr(P), n, stream_handle(stream)),
               "tsdf_import_blocks")


class Batch:
    """Several volumes advanced together by one batched step (fuse one frame
    into each, then raycast each from the same pose).  Each scene's frame
    size is fixed at creation; the step keeps per-scene vertex and normal
    maps."""

    def __init__(self, volumes: Sequence[Volume], Ks: Sequence, graph: bool = True):
        n = len(volumes)
        self.volumes = list(volumes)
        self.K = [make_intrinsics(K) for K in Ks]
        assert len(self.K) == n
        dev = self.volumes[0].buffer.device
        nbytes = int(lib().tsdf_batch_bytes(n))
        if nbytes == 0:
            raise TsdfError(EINVAL, "tsdf_batch_bytes")
        self.table = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        handles = (ctypes.c_void_p * n)(*[v.handle.value for v in self.volumes])
        intr = (Intrinsics * n)(*self.K)
        h = ctypes.c_void_p()
        _check(lib().tsdf_batch_create(handles, intr, n, _ptr(self.table), nbytes, ctypes.byref(h)),
               "tsdf_batch_create")
        self.handle = h
        self.vertex = [torch.zeros((k.height, k.width, 4), dtype=torch.float32, device=dev) for k in self.K]
        self.normal = [torch.zeros_like(v) for v in self.vertex]
        self._vp = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.vertex])
        self._np = (ctypes.c_void_p * n)(*[t.data_ptr() for t in self.normal])
        # graph capture needs a created stream; steps without an explicit one
        # run on this stream, ordered after the caller's current stream
        self.stream = torch.cuda.Stream(device=dev)
        self.set_graph(graph)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib().tsdf_batch_destroy(h)
            self.handle = None

    def set_graph(self, enable: bool):
        _check(lib().tsdf_batch_set_graph(self.handle, 1 if enable else 0), "tsdf_batch_set_graph")

    def set_persistent(self, enable: bool):
        """One cooperative launch per step instead of six (tsdf_batch.h)."""
        _check(lib().tsdf_batch_set_persistent(self.handle, 1 if enable else 0), "tsdf_batch_set_persistent")

    def set_raycast_group(self, group: int):
        _check(lib().tsdf_batch_set_raycast_group(self.handle, int(group)), "tsdf_batch_set_raycast_group")

    @property
    def raycast_group(self) -> int:
        return int(lib().tsdf_batch_get_raycast_group(self.handle))

    def _poses(self, poses) -> np.ndarray:
        arr = np.zeros((len(self.volumes), 12), np.float64)
        for k, p in enumerate(poses):
            if p is not None:
                arr[k] = _pose_array(p)
        return np.ascontiguousarray(arr)

    def step(self, depths: Sequence[Optional[torch.Tensor]], poses, noise_kind: int = NOISE_QUADRATIC,
             coeff: float = 0.0015, mlp_params: Optional[torch.Tensor] = None, stream=None):
        """depths[k] None leaves scene k untouched this step."""
        n = len(self.volumes)
        assert len(depths) == n and len(poses) == n
        dp = (ctypes.c_void_p * n)()
        for k, d in enumerate(depths):
            if d is not None:
                assert d.is_cuda and d.dtype == torch.float32 and d.is_contiguous()
                assert d.shape == (self.K[k].height, self.K[k].width)
                dp[k] = d.data_ptr()
        self._depths = list(depths)   # keep the inputs alive while the step runs
        pa = self._poses(poses)
        nm = NoiseModel(int(noise_kind), float(coeff),
                        ctypes.c_void_p(mlp_params.data_ptr()) if mlp_params is not None else None)
        own = stream is None
        if own:
            stream = self.stream
            stream.wait_stream(torch.cuda.current_stream())
        _check(lib().tsdf_batch_step(self.handle, dp, pa.ctypes.data_as(ctypes.c_void_p), self._vp, self._np,
                                     ctypes.byref(nm), stream_handle(stream)), "tsdf_batch_step")
        if own:
            torch.cuda.current_stream().wait_stream(stream)

    def autotune_raycast(self, poses, reps: int = 3, stream=None):
        pa = self._poses(poses)
        best = ctypes.c_int32(0)
        ms = ctypes.c_float(0)
        if stream is None:
            stream = self.stream
            stream.wait_stream(torch.cuda.current_stream())
        _check(lib().tsdf_batch_autotune_raycast(self.handle, pa.ctypes.data_as(ctypes.c_void_p), self._vp,
                                                 self._np, int(reps), stream_handle(stream), ctypes.byref(best),
                                                 ctypes.byref(ms)), "tsdf_batch_autotune_raycast")
        return int(best.value), float(ms.value)


    def set_fuse_grid(self, workgroups: int):
        _check(lib().tsdf_batch_set_fuse_grid(self.handle, ctypes.c_uint32(int(workgroups))), "tsdf_batch_set_fuse_grid")

    @property
    def fuse_grid(self) -> int:
        return int(lib().tsdf_batch_get_fuse_grid(self.handle))

    def autotune_fuse(self, depths: Sequence[Optional[torch.Tensor]], poses, noise_kind: int = NOISE_QUADRATIC,
                      coeff: float = 0.0015, mlp_params: Optional[torch.Tensor] = None, reps: int = 2, stream=None):
        """Picks the fusion grid by timing whole steps on these frames (which
        get fused into the volumes repeatedly: reset them afterwards)."""
        n = len(self.volumes)
        dp = (ctypes.c_void_p * n)()
        for k, d in enumerate(depths):
            if d is not None:
                assert d.is_cuda and d.dtype == torch.float32 and d.is_contiguous()
                dp[k] = d.data_ptr()
        pa = self._poses(poses)
        nm = NoiseModel(int(noise_kind), float(coeff),
                        ctypes.c_void_p(mlp_params.data_ptr()) if mlp_params is not None else None)
        best = ctypes.c_uint32(0)
        ms = ctypes.c_float(0)
        if stream is None:
            stream = self.stream
            stream.wait_stream(torch.cuda.current_stream())
        _check(lib().tsdf_batch_autotune_fuse(self.handle, dp, pa.ctypes.data_as(ctypes.c_void_p), self._vp,
                                              self._np, ctypes.byref(nm), int(reps), stream_handle(stream),
                                              ctypes.byref(best), ctypes.byref(ms)), "tsdf_batch_autotune_fuse")
        return int(best.value), float(ms.value)


class IcpParams(ctypes.Structure):
    _fields_ = [("dist_max", ctypes.c_double), ("cos_min", ctypes.c_double), ("theta", ctypes.c_double),
                ("shrink", ctypes.c_int32), ("pad", ctypes.c_int32)]


class IcpResult(ctypes.Structure):
    _fields_ = [("pose", ctypes.c_double * 12), ("x", ctypes.c_double * 6), ("lam", ctypes.c_double * 6),
                ("C", ctypes.c_double * 36), ("b", ctypes.c_double * 6), ("m", ctypes.c_double * 3),
                ("S", ctypes.c_double * 3), ("residual2", ctypes.c_double), ("pairs", ctypes.c_int64),
                ("kept", ctypes.c_int32), ("pad", ctypes.c_int32)]


ICP_RESULT_DOUBLES = ctypes.sizeof(IcpResult) // 8


class Icp:
    """Point-to-plane ICP (tsdf_icp.h) for depth maps of one size.

    Holds the device workspace and a device array of result records; the
    pose estimate stays on the device between iterations."""

    def __init__(self, K, dist_max: float = 0.02, cos_min: float = 0.9396926207859084, theta: float = 0.005,
                 shrink: bool = True, max_iters: int = 32, device: str = "cuda"):
        self.K = make_intrinsics(K)
        self.params = IcpParams(float(dist_max), float(cos_min), float(theta), 1 if shrink else 0, 0)
        nbytes = int(lib().tsdf_icp_workspace_bytes(self.K.width, self.K.height))
        if nbytes == 0:
            raise TsdfError(EINVAL, "tsdf_icp_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.results = torch.zeros((max_iters, ICP_RESULT_DOUBLES), dtype=torch.float64, device=device)

    def step(self, depth: torch.Tensor, model_vertex: torch.Tensor, model_normal: torch.Tensor, model_pose,
             pose_dev: torch.Tensor, k: int = 0, stream=None) -> torch.Tensor:
        """One iteration from the device pose `pose_dev` (12 float64); writes
        result record k and returns the device view of its pose."""
        mp = _pose_array(model_pose)
        _check(lib().tsdf_icp_step(_ptr(depth), ctypes.byref(self.K), _ptr(model_vertex), _ptr(model_normal),
                                   mp.ctypes.data_as(ctypes.c_void_p), _ptr(pose_dev), ctypes.byref(self.params),
                                   _ptr(self.workspace), ctypes.c_uint64(self.workspace.numel()),
                                   _ptr(self.results[k]), stream_handle(stream)), "tsdf_icp_step")
        return self.results[k, :12]

    def run(self, depth: torch.Tensor, model_vertex: torch.Tensor, model_normal: torch.Tensor, model_pose, pose,
            iters: int, stream=None) -> torch.Tensor:
        """`iters` chained iterations from the host pose `pose`; returns the
        device pose after the last one (record iters - 1)."""
        if not 1 <= iters <= self.results.shape[0]:
            raise ValueError("iters")
        mp, p0 = _pose_array(model_pose), _pose_array(pose)
        _check(lib().tsdf_icp_run(_ptr(depth), ctypes.byref(self.K), _ptr(model_vertex), _ptr(model_normal),
                                  mp.ctypes.data_as(ctypes.c_void_p), p0.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(self.params), int(iters), _ptr(self.workspace),
                                  ctypes.c_uint64(self.workspace.numel()), _ptr(self.results),
                                  stream_handle(stream)), "tsdf_icp_run")
        return self.results[iters - 1, :12]

    def run_noalloc(self, depth: torch.Tensor, model_vertex: torch.Tensor, model_normal: torch.Tensor, model_pose,
                    pose, iters: int, stream=None) -> torch.Tensor:
        """`run` through tsdf_icp_run_noalloc: the library's static scratch
        array instead of this object's workspace."""
        if not 1 <= iters <= self.results.shape[0]:
            raise ValueError("iters")
        mp, p0 = _pose_array(model_pose), _pose_array(pose)
        _check(lib().tsdf_icp_run_noalloc(_ptr(depth), ctypes.byref(self.K), _ptr(model_vertex), _ptr(model_normal),
                                          mp.ctypes.data_as(ctypes.c_void_p), p0.ctypes.data_as(ctypes.c_void_p),
                                          ctypes.byref(self.params), int(iters), _ptr(self.results),
                                          stream_handle(stream)), "tsdf_icp_run_noalloc")
        return self.results[iters - 1, :12]

    def result(self, k: int = 0) -> dict:
        """Record k as a dict (synchronises)."""
        raw = self.results[k].cpu().numpy().tobytes()
        r = IcpResult.from_buffer_copy(raw)
        return dict(pose=np.array(r.pose).reshape(3, 4), x=np.array(r.x), lam=np.array(r.lam),
                    C=np.array(r.C).reshape(6, 6), b=np.array(r.b), m=np.array(r.m), S=np.array(r.S),
                    residual2=r.residual2, N=int(r.pairs), kept=int(r.kept))

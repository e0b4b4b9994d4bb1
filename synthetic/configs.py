"""The synthetic workloads: grids, cameras, sequences and their seeds.

  c1  one 160x120 frame of a sphere (r 0.3 m, 1 m ahead), 128^3 grid of 5 mm
  c2  100 frames of 640x480 orbiting a ground plane with 20 spheres/boxes,
      2048^3 grid of 1 mm voxels, hash capacity 2^20 blocks
  c3  300 frames of 1280x960 around a 15 cm capsule hand at 0.3-0.5 m,
      4096^3 grid of 0.15 mm voxels
  c5  16 scenes of uneven size: grids 500^3-3000^3 in a 3 m box, frames
      320x240-640x480, 30-120 frames each

All of them use the sensor model sigma = 0.0015 z^2 (Gaussian); c2 and c5
add 2 % dropout near depth edges.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Tuple

import numpy as np
import torch

from .scenes import (Intrinsics, Scene, hand_scene, look_at, procedural_scene, sensor_depth,
                     sphere_scene)


@dataclasses.dataclass(frozen=True)
class GridSpec:
    dims: Tuple[int, int, int]        # voxels per axis, each a multiple of 8
    voxel_size: float                 # metres
    origin: Tuple[float, float, float]  # min corner of the grid, metres
    trunc_voxels: float = 4.0
    capacity_blocks: int = 1 << 16
    hash_slots: int = 1 << 17

    @property
    def delta(self) -> float:
        return self.trunc_voxels * self.voxel_size


@dataclasses.dataclass
class SequenceSpec:
    name: str
    grid: GridSpec
    K: Intrinsics
    scene: Scene
    poses: List[np.ndarray]
    noise_seeds: List[Optional[int]]
    dropout_seeds: List[Optional[int]]
    near: float = 0.0
    far: float = math.inf

    @property
    def n_frames(self) -> int:
        return len(self.poses)


def sequence_frame(spec: SequenceSpec, k: int, device="cpu") -> Tuple[torch.Tensor, np.ndarray]:
    """Depth map (float32 [H, W], metres) and camera-to-world pose of frame k."""
    d = sensor_depth(spec.scene, spec.K, spec.poses[k], spec.noise_seeds[k], spec.near,
                     spec.far, spec.dropout_seeds[k], device)
    return d, spec.poses[k]


def round_up8(n: int) -> int:
    return 8 * int(math.ceil(n / 8))


def config_c1(noise: bool = True) -> SequenceSpec:
    K = Intrinsics(150.0, 150.0, 80.0, 60.0, 160, 120)
    grid = GridSpec((128, 128, 128), 0.005, (-0.32, -0.32, 0.68), 4.0, 4096, 8192)
    pose = np.hstack([np.eye(3), np.zeros((3, 1))])
    return SequenceSpec("c1-sphere-160x120", grid, K, sphere_scene((0.0, 0.0, 1.0), 0.3), [pose],
                        [1 if noise else None], [None])


def orbit_poses(n: int, radius=1.2, height=0.8, target=(0.0, 0.0, 0.0), turns=1.0) -> List[np.ndarray]:
    out = []
    for k in range(n):
        a = 2 * math.pi * turns * k / n
        eye = (radius * math.cos(a), height, radius * math.sin(a))
        out.append(look_at(eye, target))
    return out


def config_c2(n_frames: int = 100, scene_seed: int = 2, noise: bool = True, dropout: bool = True,
              width: int = 640, height: int = 480) -> SequenceSpec:
    f = 525.0 * width / 640.0
    K = Intrinsics(f, f, width / 2.0, height / 2.0, width, height)
    grid = GridSpec((2048, 2048, 2048), 0.001, (-1.024, -0.1, -1.024), 4.0, 1 << 20, 1 << 21)
    poses = orbit_poses(n_frames)
    ns = [1000 + k if noise else None for k in range(n_frames)]
    ds = [5000 + k if dropout else None for k in range(n_frames)]
    return SequenceSpec(f"c2-orbit-{width}x{height}", grid, K, procedural_scene(scene_seed), poses,
                        ns, ds, 0.3, 4.0)


def hand_poses(n: int, centre) -> List[np.ndarray]:
    out = []
    c = np.asarray(centre, np.float64)
    for k in range(n):
        ph = 2 * math.pi * k / n
        az = (math.pi / 3) * math.sin(ph)
        el = (math.pi / 6) * math.sin(2 * ph)
        rng = 0.4 + 0.1 * math.sin(ph)
        eye = c + rng * np.array([math.cos(el) * math.sin(az), math.sin(el),
                                  math.cos(el) * math.cos(az)])
        out.append(look_at(eye, c))
    return out


def config_c3(n_frames: int = 300, scene_seed: int = 3, noise: bool = True,
              width: int = 1280, height: int = 960) -> SequenceSpec:
    f = 1400.0 * width / 1280.0
    K = Intrinsics(f, f, width / 2.0, height / 2.0, width, height)
    scene = hand_scene(scene_seed)
    c = scene.centre()
    G = 4096
    vs = 0.00015
    origin = tuple(float(x) for x in (c - 0.5 * G * vs))
    grid = GridSpec((G, G, G), vs, origin, 4.0, 1 << 18, 1 << 19)
    poses = hand_poses(n_frames, c)
    ns = [3000 + k if noise else None for k in range(n_frames)]
    return SequenceSpec(f"c3-hand-{width}x{height}", grid, K, scene, poses, ns,
                        [None] * n_frames, 0.1, 2.0)


def c5_layout() -> List[dict]:
    """Per-scene sizes of the 16-scene batch: grid, voxel size, frame size, frame count."""
    G = [round_up8(int(round(g))) for g in np.linspace(500, 3000, 16)]
    counts = np.round(np.linspace(30, 120, 16)).astype(int)
    perm = np.random.default_rng(399).permutation(16)
    counts = counts[perm]
    sizes = [(320, 240), (480, 360), (640, 480)]
    out = []
    for s in range(16):
        W, H = sizes[s % 3]
        vs = 3.0 / G[s]
        # a 3 m ground plane plus objects: about 9e5 blocks at 1 mm, scaling with the area in blocks
        cap = 1 << int(math.ceil(math.log2(max(4096, 900000 * (0.001 / vs) ** 2))))
        out.append(dict(G=G[s], vs=vs, W=W, H=H, frames=int(counts[s]), capacity=min(cap, 1 << 20)))
    return out


def config_c5(scene_index: int, frame_limit: Optional[int] = None) -> SequenceSpec:
    lay = c5_layout()[scene_index]
    W, H = lay["W"], lay["H"]
    f = 525.0 * W / 640.0
    K = Intrinsics(f, f, W / 2.0, H / 2.0, W, H)
    G = lay["G"]
    cap = lay["capacity"]
    grid = GridSpec((G, G, G), lay["vs"], (-1.5, -0.1, -1.5), 4.0, cap, 2 * cap)
    n = lay["frames"] if frame_limit is None else min(frame_limit, lay["frames"])
    poses = orbit_poses(lay["frames"])[:n]
    seed = 300 + scene_index
    ns = [10000 * (scene_index + 1) + k for k in range(n)]
    ds = [20000 * (scene_index + 1) + k for k in range(n)]
    return SequenceSpec(f"c5-scene{scene_index}-{W}x{H}-G{G}", grid, K, procedural_scene(seed),
                        poses, ns, ds, 0.3, 4.0)


def small_orbit(width=80, height=60, n_frames=4, G=256, vs=0.008, seed=2) -> SequenceSpec:
    """A reduced c2-style sequence small enough for the oracle in tests."""
    f = 525.0 * width / 640.0
    K = Intrinsics(f, f, width / 2.0, height / 2.0, width, height)
    half = 0.5 * G * vs
    grid = GridSpec((G, G, G), vs, (-half, -0.1, -half), 4.0, 1 << 15, 1 << 16)
    poses = orbit_poses(n_frames)
    return SequenceSpec(f"small-orbit-{width}x{height}-G{G}", grid, K, procedural_scene(seed),
                        poses, [1000 + k for k in range(n_frames)],
                        [5000 + k for k in range(n_frames)], 0.3, 4.0)

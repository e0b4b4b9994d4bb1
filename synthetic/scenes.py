"""Analytic scenes and depth rendering in float64.

Conventions (shared with every consumer of these inputs):
  * A pose is camera-to-world, a 3x4 row-major float64 matrix [R | t]:
    x_world = R @ x_cam + t.
  * Camera axes: x right, y down, z forward.  Pixel (i, j) is column i,
    row j, and its centre sits at image coordinates (u, v) = (i, j), so the
    ray through it has camera direction ((i - cx)/fx, (j - cy)/fy, 1).
  * A depth map D[j, i] holds the camera-z distance in metres, 0 where the
    ray hits nothing or falls outside the sensor range.

Scenes are unions of solids.  Each primitive offers a ray entry distance
(first intersection) and a signed distance (positive outside).  Rendering
takes the nearest entry over all primitives, which is exact for a union of
solids seen from outside every solid.

Everything here works on any torch device; the randomness (scene layout,
noise, dropout) always comes from CPU generators so that a given seed gives
the same scene and the same noise on every machine.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

F64 = torch.float64


@dataclasses.dataclass(frozen=True)
class Intrinsics:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def as_tuple(self):
        return (self.fx, self.fy, self.cx, self.cy, self.width, self.height)


@dataclasses.dataclass
class Scene:
    """A union of solids.

    spheres:  [n, 4]  (cx, cy, cz, r)
    boxes:    [n, 7]  (cx, cy, cz, hx, hy, hz, yaw)   yaw about +y
    capsules: [n, 7]  (ax, ay, az, bx, by, bz, r)
    planes:   [n, 4]  (nx, ny, nz, h): solid where n.x < h, n unit
    """

    spheres: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 4)))
    boxes: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 7)))
    capsules: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 7)))
    planes: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 4)))

    def centre(self) -> np.ndarray:
        pts = []
        if len(self.spheres):
            pts.append(self.spheres[:, :3])
        if len(self.boxes):
            pts.append(self.boxes[:, :3])
        if len(self.capsules):
            pts.append(0.5 * (self.capsules[:, :3] + self.capsules[:, 3:6]))
        if not pts:
            return np.zeros(3)
        allp = np.concatenate(pts, 0)
        return 0.5 * (allp.min(0) + allp.max(0))


# ---------------------------------------------------------------------------
# Camera paths


def look_at(eye: Sequence[float], target: Sequence[float], up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """Camera-to-world pose looking from eye at target, camera y pointing down.

    The camera frame is right-handed (x right, y down, z forward), so
    right = forward x up and down = forward x right.
    """
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f = f / np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r = r / np.linalg.norm(r)
    d = np.cross(f, r)
    pose = np.zeros((3, 4))
    pose[:, 0] = r
    pose[:, 1] = d
    pose[:, 2] = f
    pose[:, 3] = eye
    return pose


# ---------------------------------------------------------------------------
# Ray / primitive entry distances.  Rays are o + lam * d with d in world
# units; lam is returned (inf where there is no entry with lam > 0).


def _nearest_positive(r0, r1):
    inf = torch.full_like(r0, math.inf)
    r0 = torch.where(torch.isfinite(r0) & (r0 > 0), r0, inf)
    r1 = torch.where(torch.isfinite(r1) & (r1 > 0), r1, inf)
    return torch.minimum(r0, r1)


def _ray_sphere(o, d, c, r):
    oc = o - c
    a = (d * d).sum(-1)
    b = (d * oc).sum(-1)
    c0 = (oc * oc).sum(-1) - r * r
    disc = b * b - a * c0
    ok = disc >= 0
    sq = torch.sqrt(torch.clamp(disc, min=0.0))
    r0 = (-b - sq) / a
    r1 = (-b + sq) / a
    lam = _nearest_positive(r0, r1)
    return torch.where(ok, lam, torch.full_like(lam, math.inf))


def _ray_plane(o, d, n, h):
    nd = (d * n).sum(-1)
    no = (o * n).sum(-1)
    lam = (h - no) / nd
    ok = (nd != 0) & (lam > 0)
    return torch.where(ok, lam, torch.full_like(lam, math.inf))


def _yaw_matrix(yaw, dev):
    c, s = math.cos(yaw), math.sin(yaw)
    return torch.tensor([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]], dtype=F64, device=dev)


def _ray_box(o, d, centre, half, yaw):
    Ry = _yaw_matrix(yaw, o.device)
    ol = (o - centre) @ Ry  # = Ry^T (o - c) row-wise
    dl = d @ Ry
    with torch.no_grad():
        inv = 1.0 / dl
        t1 = (-half - ol) * inv
        t2 = (half - ol) * inv
        tmin = torch.minimum(t1, t2).amax(-1)
        tmax = torch.maximum(t1, t2).amin(-1)
    ok = (tmax >= tmin) & (tmax > 0)
    lam = torch.where(tmin > 0, tmin, tmax)
    return torch.where(ok, lam, torch.full_like(lam, math.inf))


def _ray_capsule(o, d, a, b, r):
    """Entry into the union of two end spheres and the lateral cylinder.

    The flat discs closing the finite cylinder lie inside the end spheres,
    so the first entry into the capsule is the smallest of: the two sphere
    entries and the lateral-surface entries whose axial coordinate lies on
    the segment.
    """
    lam = torch.minimum(_ray_sphere(o, d, a, r), _ray_sphere(o, d, b, r))
    axis = b - a
    L = float(torch.linalg.norm(axis))
    w = axis / L
    m = o - a
    dw = (d * w).sum(-1, keepdim=True)
    mw = (m * w).sum(-1, keepdim=True)
    dp = d - dw * w
    mp = m - mw * w
    A = (dp * dp).sum(-1)
    B = (dp * mp).sum(-1)
    C = (mp * mp).sum(-1) - r * r
    disc = B * B - A * C
    ok = (disc >= 0) & (A > 0)
    sq = torch.sqrt(torch.clamp(disc, min=0.0))
    Asafe = torch.where(A > 0, A, torch.ones_like(A))
    for root in ((-B - sq) / Asafe, (-B + sq) / Asafe):
        ax = mw[..., 0] + root * dw[..., 0]
        good = ok & (root > 0) & (ax >= 0) & (ax <= L)
        lam = torch.where(good, torch.minimum(lam, root), lam)
    return lam


def ray_entry(scene: Scene, o: torch.Tensor, d: torch.Tensor) -> torch.Tensor:
    """Nearest entry parameter of rays o + lam d into the scene (inf: miss)."""
    dev = d.device
    lam = torch.full(d.shape[:-1], math.inf, dtype=F64, device=dev)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), dtype=F64, device=dev)  # noqa: E731
    for s in scene.spheres:
        lam = torch.minimum(lam, _ray_sphere(o, d, t(s[:3]), float(s[3])))
    for p in scene.planes:
        lam = torch.minimum(lam, _ray_plane(o, d, t(p[:3]), float(p[3])))
    for bx in scene.boxes:
        lam = torch.minimum(lam, _ray_box(o, d, t(bx[:3]), t(bx[3:6]), float(bx[6])))
    for c in scene.capsules:
        lam = torch.minimum(lam, _ray_capsule(o, d, t(c[:3]), t(c[3:6]), float(c[6])))
    return lam


def pixel_rays(K: Intrinsics, pose: np.ndarray, device="cpu"):
    """World-space rays through pixel centres; d has camera-z component 1."""
    dev = torch.device(device)
    i = torch.arange(K.width, dtype=F64, device=dev)
    j = torch.arange(K.height, dtype=F64, device=dev)
    jj, ii = torch.meshgrid(j, i, indexing="ij")
    dc = torch.stack([(ii - K.cx) / K.fx, (jj - K.cy) / K.fy, torch.ones_like(ii)], -1)
    R = torch.as_tensor(pose[:, :3], dtype=F64, device=dev)
    tvec = torch.as_tensor(pose[:, 3], dtype=F64, device=dev)
    d = dc @ R.T
    o = tvec.expand_as(d)
    return o, d


def render_depth(scene: Scene, K: Intrinsics, pose: np.ndarray, near=0.0, far=math.inf,
                 device="cpu") -> torch.Tensor:
    """Noise-free camera-z depth [H, W] float64; 0 = no return."""
    o, d = pixel_rays(K, pose, device)
    lam = ray_entry(scene, o, d)
    ok = torch.isfinite(lam) & (lam >= near) & (lam <= far)
    return torch.where(ok, lam, torch.zeros_like(lam))


def render_model_maps(scene: Scene, K: Intrinsics, pose: np.ndarray, near=0.0, far=math.inf, eps=1e-6):
    """Exact vertex and normal maps of the scene seen from `pose`, in the
    layout a raycast produces: float32 [H, W, 4] each, world coordinates,
    w = 1 where the pixel's ray hits a surface and 0 elsewhere.  The normal
    is the normalised central-difference gradient of the scene's signed
    distance (step eps metres), so it faces out of the solids."""
    o, d = pixel_rays(K, pose)
    lam = ray_entry(scene, o, d)
    zc = lam   # d has camera-z component 1, so lam is the camera depth
    ok = torch.isfinite(lam) & (zc >= near) & (zc <= far)
    x = o + torch.where(ok, lam, torch.zeros_like(lam))[..., None] * d
    g = torch.zeros_like(x)
    for a in range(3):
        e = torch.zeros(3, dtype=F64)
        e[a] = eps
        g[..., a] = scene_sdf(scene, x + e) - scene_sdf(scene, x - e)
    g = g / torch.linalg.norm(g, dim=-1, keepdim=True).clamp_min(1e-300)
    w = ok.to(F64)[..., None]
    vert = torch.cat([x * w, w], -1).to(torch.float32)
    nrm = torch.cat([g * w, w], -1).to(torch.float32)
    return vert, nrm


# ---------------------------------------------------------------------------
# Signed distances (positive outside) for ground truth.


def scene_sdf(scene: Scene, x: torch.Tensor) -> torch.Tensor:
    """Signed distance of the union at points x [..., 3] (float64)."""
    dev = x.device
    t = lambda a: torch.as_tensor(np.asarray(a, np.float64), dtype=F64, device=dev)  # noqa: E731
    out = torch.full(x.shape[:-1], math.inf, dtype=F64, device=dev)
    for s in scene.spheres:
        out = torch.minimum(out, torch.linalg.norm(x - t(s[:3]), dim=-1) - float(s[3]))
    for p in scene.planes:
        out = torch.minimum(out, (x * t(p[:3])).sum(-1) - float(p[3]))
    for bx in scene.boxes:
        Ry = _yaw_matrix(float(bx[6]), dev)
        q = ((x - t(bx[:3])) @ Ry).abs() - t(bx[3:6])
        outside = torch.linalg.norm(torch.clamp(q, min=0.0), dim=-1)
        inside = torch.clamp(q.amax(-1), max=0.0)
        out = torch.minimum(out, outside + inside)
    for c in scene.capsules:
        a, b, r = t(c[:3]), t(c[3:6]), float(c[6])
        ab = b - a
        h = torch.clamp(((x - a) * ab).sum(-1) / (ab * ab).sum(), 0.0, 1.0)
        out = torch.minimum(out, torch.linalg.norm(x - a - h[..., None] * ab, dim=-1) - r)
    return out


# ---------------------------------------------------------------------------
# Scene builders


def sphere_scene(centre=(0.0, 0.0, 1.0), radius=0.3) -> Scene:
    return Scene(spheres=np.array([[*centre, radius]], np.float64))


def plane_scene(normal, h) -> Scene:
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    return Scene(planes=np.array([[*n, h]], np.float64))


def procedural_scene(seed: int, n_objects=20, disc_radius=0.7, size_range=(0.05, 0.40)) -> Scene:
    """Ground plane y = 0 plus alternating spheres and yawed boxes resting on it.

    Object sizes are uniform in size_range (sphere diameter, box edge);
    centres are uniform in a disc of disc_radius around the origin.
    """
    rng = np.random.default_rng(seed)
    spheres, boxes = [], []
    for k in range(n_objects):
        size = rng.uniform(*size_range)
        rad = disc_radius * math.sqrt(rng.uniform())
        ang = rng.uniform(0, 2 * math.pi)
        px, pz = rad * math.cos(ang), rad * math.sin(ang)
        if k % 2 == 0:
            r = 0.5 * size
            spheres.append([px, r, pz, r])
        else:
            hx = 0.5 * size
            hy = 0.5 * size * rng.uniform(0.5, 1.0)
            hz = 0.5 * size * rng.uniform(0.6, 1.0)
            boxes.append([px, hy, pz, hx, hy, hz, rng.uniform(0, math.pi)])
    return Scene(spheres=np.array(spheres, np.float64).reshape(-1, 4),
                 boxes=np.array(boxes, np.float64).reshape(-1, 7),
                 planes=np.array([[0.0, 1.0, 0.0, 0.0]], np.float64))


def hand_scene(seed: int, centre=(0.0, 0.0, 0.0)) -> Scene:
    """A hand-like union of capsules, about 15 cm long, palm facing +z.

    Palm: 3-4 transverse capsules of radius 12-15 mm.  Five fingers (the
    thumb on the side) of 2-3 phalanx capsules of radius 7-9 mm whose joint
    angles bend each finger towards -z by a seeded amount.
    """
    rng = np.random.default_rng(seed)
    c = np.asarray(centre, np.float64)
    caps = []
    n_palm = int(rng.integers(3, 5))
    palm_w, palm_h = 0.070, 0.075
    y0 = -0.065
    for k in range(n_palm):
        y = y0 + (k + 0.5) * palm_h / n_palm
        r = rng.uniform(0.012, 0.015)
        caps.append([-0.5 * palm_w + r, y, 0.0, 0.5 * palm_w - r, y, 0.0, r])
    top = y0 + palm_h
    xs = np.linspace(-0.027, 0.027, 4)
    lengths = [0.060, 0.068, 0.064, 0.050]
    for x, L in zip(xs, lengths):
        nseg = int(rng.integers(2, 4))
        r = rng.uniform(0.007, 0.009)
        p = np.array([x, top - 0.005, 0.0])
        ang = 0.0
        for s in range(nseg):
            ang += rng.uniform(0.05, 0.35)
            seg = L / nseg
            q = p + seg * np.array([0.0, math.cos(ang), -math.sin(ang)])
            caps.append([*p, *q, r])
            p = q
    # thumb from the lower side of the palm, pointing outwards and up
    p = np.array([-0.5 * palm_w + 0.005, y0 + 0.02, 0.0])
    r = rng.uniform(0.008, 0.009)
    nseg = int(rng.integers(2, 4))
    ang = rng.uniform(0.5, 0.9)
    for s in range(nseg):
        seg = 0.055 / nseg
        q = p + seg * np.array([-math.sin(ang), math.cos(ang), -0.2])
        caps.append([*p, *q, r])
        p = q
        ang -= rng.uniform(0.1, 0.3)
    caps = np.array(caps, np.float64)
    caps[:, :3] += c
    caps[:, 3:6] += c
    return Scene(capsules=caps)


# ---------------------------------------------------------------------------
# Sensor model


def add_sensor_noise(depth: torch.Tensor, seed: int, coeff=0.0015) -> torch.Tensor:
    """D + coeff * D^2 * N(0, 1) on valid pixels; invalid pixels stay 0."""
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    eps = torch.randn(depth.shape, generator=g, dtype=F64).to(depth.device)
    noisy = depth + coeff * depth * depth * eps
    return torch.where(depth > 0, noisy, torch.zeros_like(depth))


def depth_discontinuities(depth: torch.Tensor, rel=0.05) -> torch.Tensor:
    """Valid pixels with a 4-neighbour jump |dD| > rel * D or an invalid 4-neighbour.

    Neighbours outside the image do not count.
    """
    D = depth
    H, W = D.shape
    valid = D > 0
    disc = torch.zeros_like(valid)
    for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
        nb = torch.zeros_like(D)
        inb = torch.zeros_like(valid)
        js = slice(max(dj, 0), H + min(dj, 0))
        jd = slice(max(-dj, 0), H + min(-dj, 0))
        is_ = slice(max(di, 0), W + min(di, 0))
        id_ = slice(max(-di, 0), W + min(-di, 0))
        nb[jd, id_] = D[js, is_]
        inb[jd, id_] = True
        jump = (nb <= 0) | ((nb - D).abs() > rel * D)
        disc |= valid & inb & jump
    return disc


def edge_dropout(clean: torch.Tensor, noisy: torch.Tensor, seed: int, frac=0.02,
                 radius=2) -> torch.Tensor:
    """Zero round(frac*W*H) pixels drawn from those within `radius` px of a discontinuity.

    Distance is Chebyshev (a (2r+1)^2 window) and discontinuities are found
    on the clean depth.  If fewer candidates exist, all of them drop out.
    """
    H, W = clean.shape
    disc = depth_discontinuities(clean).to(torch.float32)[None, None]
    near = torch.nn.functional.max_pool2d(disc, 2 * radius + 1, stride=1, padding=radius)[0, 0] > 0
    near &= clean > 0
    idx = torch.nonzero(near.flatten().cpu()).flatten()
    n = min(int(round(frac * W * H)), idx.numel())
    g = torch.Generator(device="cpu").manual_seed(int(seed))
    pick = idx[torch.randperm(idx.numel(), generator=g)[:n]]
    out = noisy.clone().flatten()
    out[pick.to(out.device)] = 0.0
    return out.view(H, W)


def sensor_depth(scene: Scene, K: Intrinsics, pose: np.ndarray, noise_seed: Optional[int],
                 near=0.0, far=math.inf, dropout_seed: Optional[int] = None,
                 device="cpu") -> torch.Tensor:
    """Rendered depth with optional Gaussian noise and edge dropout, float32 [H, W]."""
    clean = render_depth(scene, K, pose, near, far, device)
    d = clean if noise_seed is None else add_sensor_noise(clean, noise_seed)
    if dropout_seed is not None:
        d = edge_dropout(clean, d, dropout_seed)
    return d.to(torch.float32)


def ensure_list(x) -> List:
    return list(x) if isinstance(x, (list, tuple)) else [x]

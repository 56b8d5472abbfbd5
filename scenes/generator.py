"""Seeded synthetic point clouds standing in for the paper's sampled clouds.

The paper renders 2^23 view-specific samples per training iteration
(Sec. 2, "A Note on Sample Count") and 33-67 M pre-extracted points
(Sec. 3.1 and Tab. 4) at 1-2 megapixels, with four features per point
(Sec. 2, "Implicit Point Cloud").  Its scenes (Mip-NeRF360, Tanks and
Temples) are not available, so these generators draw clouds with the same
structure: most points concentrated on a few surfaces, the rest spread
through a box in front of a pinhole camera.

Draw order for one scene (fixed, so a seed pins every value):
  1. surface parameters   2. surface points (+ jitter)   3. uniform points
  4. opacity   5. features   5b. Gaussian radii (only when requested)
  6. upstream gradient (only when requested)   7. a shuffle of point order
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

Z_NEAR_DEFAULT = 0.2


@dataclasses.dataclass
class Camera:
    """Pinhole camera, OpenCV axes (+z forward, +y down).

    A world point p maps to camera space as X = R p + t (R row-major).
    """

    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # (3, 3) float32
    t: np.ndarray  # (3,) float32
    z_near: float = Z_NEAR_DEFAULT

    def as_tuple(self):
        return (self.width, self.height, self.fx, self.fy, self.cx, self.cy,
                tuple(float(x) for x in np.asarray(self.R, np.float32).reshape(-1)),
                tuple(float(x) for x in np.asarray(self.t, np.float32).reshape(-1)),
                self.z_near)


@dataclasses.dataclass
class SceneSpec:
    n: int
    s: float = 1.0
    z_lo: float = 2.0
    z_hi: float = 6.0
    width: int = 256
    height: int = 256
    focal: Optional[float] = None  # default: width / 2 (90 degree horizontal FOV)
    channels: int = 4
    feat_dist: str = "uniform01"  # or "normal"
    opacity_range: Tuple[float, float] = (0.1, 0.9)
    radius_range: Optional[Tuple[float, float]] = None  # Gaussian splats only
    with_grad: bool = False
    with_grad_t: bool = False
    seed: int = 0


@dataclasses.dataclass
class Scene:
    pos: np.ndarray  # (N, 3) float32
    opacity: np.ndarray  # (N,) float32
    feat: np.ndarray  # (N, C) float32
    camera: Camera
    radius: Optional[np.ndarray] = None  # (N,) float32
    grad: Optional[np.ndarray] = None  # (C, H, W) float32
    grad_t: Optional[np.ndarray] = None  # (H, W) float32
    spec: Optional[SceneSpec] = None

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    @property
    def channels(self) -> int:
        return int(self.feat.shape[1])


def make_camera(width: int, height: int, focal: Optional[float] = None,
                z_near: float = Z_NEAR_DEFAULT) -> Camera:
    """Camera at the origin looking down +z, principal point at the image centre."""
    f = float(width) / 2.0 if focal is None else float(focal)
    return Camera(width=int(width), height=int(height), fx=f, fy=f,
                  cx=width / 2.0, cy=height / 2.0,
                  R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32),
                  z_near=z_near)


def ring_camera(view: int, n_views: int, width: int, height: int,
                radius: float = 8.0, centre=(0.0, 0.0, 11.0),
                z_near: float = Z_NEAR_DEFAULT) -> Camera:
    """Camera on a horizontal ring around `centre`, looking at it.

    View v sits at angle 2*pi*v/n_views; angle 0 is centre - radius * z,
    looking down +z, so view 0 equals the default camera moved to z = 3.
    """
    th = 2.0 * math.pi * view / n_views
    c = np.asarray(centre, np.float64)
    eye = c + radius * np.array([math.sin(th), 0.0, -math.cos(th)])
    z_axis = (c - eye) / np.linalg.norm(c - eye)
    y_axis = np.array([0.0, 1.0, 0.0])
    x_axis = np.cross(y_axis, z_axis)
    R = np.stack([x_axis, y_axis, z_axis]).astype(np.float64)
    t = -R @ eye
    f = float(width) / 2.0
    return Camera(width=int(width), height=int(height), fx=f, fy=f,
                  cx=width / 2.0, cy=height / 2.0,
                  R=R.astype(np.float32), t=t.astype(np.float32), z_near=z_near)


def _plane_basis(nrm: np.ndarray):
    a = np.zeros(3)
    a[int(np.argmin(np.abs(nrm)))] = 1.0
    e1 = np.cross(nrm, a)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(nrm, e1)
    return e1, e2


def draw_surfaces(rng: np.random.Generator, s: float, z_lo: float, z_hi: float):
    """Step 1: four surfaces (planes k=0,2; spheres k=1,3) with centres in the
    box shrunk 25% toward its centre."""
    lo = np.array([-s, -s, z_lo])
    hi = np.array([s, s, z_hi])
    mid = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    s_lo, s_hi = mid - 0.75 * half, mid + 0.75 * half
    surfaces = []
    for k in range(4):
        centre = rng.uniform(s_lo, s_hi)
        if k % 2 == 0:
            nrm = rng.normal(size=3)
            nrm /= np.linalg.norm(nrm)
            surfaces.append(("plane", centre, nrm))
        else:
            surfaces.append(("sphere", centre, rng.uniform(0.1, 0.25) * s))
    return surfaces


def draw_points(rng: np.random.Generator, n: int, s: float, z_lo: float,
                z_hi: float, surfaces=None) -> np.ndarray:
    """Steps 1-3: four surfaces (drawn here unless given) plus uniform points."""
    lo = np.array([-s, -s, z_lo])
    hi = np.array([s, s, z_hi])
    if surfaces is None:
        surfaces = draw_surfaces(rng, s, z_lo, z_hi)
    n_surf = int(0.7 * n)
    counts = [n_surf // 4] * 4
    counts[3] += n_surf - sum(counts)
    parts = []
    for (kind, centre, prm), cnt in zip(surfaces, counts):  # step 2
        if kind == "plane":
            e1, e2 = _plane_basis(prm)
            ab = rng.uniform(-0.5, 0.5, size=(cnt, 2)) * s
            p = centre + ab[:, :1] * e1 + ab[:, 1:] * e2
        else:
            d = rng.normal(size=(cnt, 3))
            d /= np.linalg.norm(d, axis=1, keepdims=True)
            p = centre + prm * d
        p = p + rng.normal(0.0, 0.01 * s, size=(cnt, 3))
        parts.append(p)
    parts.append(rng.uniform(lo, hi, size=(n - n_surf, 3)))  # step 3
    return np.concatenate(parts, axis=0)


def make_scene(spec: SceneSpec, camera: Optional[Camera] = None, rng=None,
               surfaces=None) -> Scene:
    rng = np.random.default_rng(spec.seed) if rng is None else rng
    pos = draw_points(rng, spec.n, spec.s, spec.z_lo, spec.z_hi, surfaces)
    lo, hi = spec.opacity_range
    opacity = rng.uniform(lo, hi, size=spec.n)  # step 4
    if spec.feat_dist == "uniform01":  # step 5
        feat = rng.uniform(0.0, 1.0, size=(spec.n, spec.channels))
    elif spec.feat_dist == "normal":
        feat = rng.standard_normal(size=(spec.n, spec.channels))
    else:
        raise ValueError(spec.feat_dist)
    radius = None
    if spec.radius_range is not None:  # step 5b
        radius = rng.uniform(spec.radius_range[0], spec.radius_range[1], size=spec.n)
    cam = camera if camera is not None else make_camera(spec.width, spec.height, spec.focal)
    grad = grad_t = None
    if spec.with_grad:  # step 6
        grad = rng.standard_normal(size=(spec.channels, cam.height, cam.width)).astype(np.float32)
    if spec.with_grad_t:
        grad_t = rng.standard_normal(size=(cam.height, cam.width)).astype(np.float32)
    perm = rng.permutation(spec.n)  # step 7
    pos = np.ascontiguousarray(pos[perm], dtype=np.float32)
    opacity = np.ascontiguousarray(opacity[perm], dtype=np.float32)
    feat = np.ascontiguousarray(feat[perm], dtype=np.float32)
    if radius is not None:
        radius = np.ascontiguousarray(radius[perm], dtype=np.float32)
    return Scene(pos=pos, opacity=opacity, feat=feat, camera=cam, radius=radius,
                 grad=grad, grad_t=grad_t, spec=spec)


def tiny_scene(n: int, width: int, height: int, channels: int = 3, seed: int = 0,
               focal: Optional[float] = None, z_range=(2.0, 4.0), spread: float = 1.0,
               opacity_range=(0.05, 0.95), radius_range=None, with_grad: bool = True,
               with_grad_t: bool = False) -> Scene:
    """A small uniform cloud in the view frustum, for brute-force checks."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(z_range[0], z_range[1], size=n)
    f = float(width) / 2.0 if focal is None else float(focal)
    # spread slightly beyond the image so border handling is exercised
    xn = rng.uniform(-spread, spread, size=n) * (width / 2.0 + 2.0) / f
    yn = rng.uniform(-spread, spread, size=n) * (height / 2.0 + 2.0) / f
    pos = np.stack([xn * z, yn * z, z], axis=1)
    opacity = rng.uniform(opacity_range[0], opacity_range[1], size=n)
    feat = rng.standard_normal(size=(n, channels))
    radius = None
    if radius_range is not None:
        radius = rng.uniform(radius_range[0], radius_range[1], size=n).astype(np.float32)
    cam = make_camera(width, height, f)
    grad = rng.standard_normal(size=(channels, height, width)).astype(np.float32) if with_grad else None
    grad_t = rng.standard_normal(size=(height, width)).astype(np.float32) if with_grad_t else None
    return Scene(pos=pos.astype(np.float32), opacity=opacity.astype(np.float32),
                 feat=feat.astype(np.float32), camera=cam, radius=radius, grad=grad,
                 grad_t=grad_t)


# Workload configurations.  Sizes use powers of two where the paper counts
# samples that way (2^21, 2^23, 2^24); other counts are decimal.
CONFIGS = {
    # plain FP32 forward, correctness size
    "C1": SceneSpec(n=50_000, s=1.0, z_lo=2.0, z_hi=6.0, width=256, height=256, focal=256.0,
                    channels=4, feat_dist="uniform01", opacity_range=(0.1, 0.9), seed=0),
    # plain FP32 forward + backward, 720p
    "C2": SceneSpec(n=2 ** 21, s=4.0, z_lo=2.0, z_hi=20.0, width=1280, height=720,
                    channels=16, feat_dist="normal", opacity_range=(0.05, 0.95),
                    with_grad=True, seed=0),
    # headline: 2^23 points, 1080p, forward + backward
    "H": SceneSpec(n=2 ** 23, s=4.0, z_lo=2.0, z_hi=20.0, width=1920, height=1080,
                   channels=16, feat_dist="normal", opacity_range=(0.05, 0.95),
                   with_grad=True, seed=0),
    # inference Gaussians, forward only
    "C3": SceneSpec(n=2 ** 23, s=4.0, z_lo=2.0, z_hi=20.0, width=1920, height=1080,
                    channels=16, feat_dist="normal", opacity_range=(0.05, 0.95),
                    radius_range=(0.5, 3.0), seed=0),
    # mixed precision, 2^24 points, 32 channels
    "C5": SceneSpec(n=2 ** 24, s=4.0, z_lo=2.0, z_hi=20.0, width=1920, height=1080,
                    channels=32, feat_dist="normal", opacity_range=(0.05, 0.95),
                    with_grad=True, seed=0),
}


# Multi-view batch: 8 views of one scene (the four surfaces of seed 0 in the
# box [-4, 4]^2 x [2, 20]), each with its own point sample of n_v ~ U{500,000
# .. 6,000,000} points (seed (0, v)) and a resolution drawn from {960x540,
# 1280x720, 1920x1080}; cameras on a ring of radius 8 around the box centre.
MULTI_VIEW_RESOLUTIONS = ((960, 540), (1280, 720), (1920, 1080))


def multi_view_specs(n_views: int = 8, seed: int = 0, n_lo: int = 500_000,
                     n_hi: int = 6_000_000, channels: int = 16, resolutions=None):
    """Per-view (SceneSpec, Camera) pairs of the multi-view batch."""
    res = MULTI_VIEW_RESOLUTIONS if resolutions is None else tuple(resolutions)
    cfg = np.random.default_rng(seed)
    counts = cfg.integers(n_lo, n_hi + 1, size=n_views)
    picks = cfg.integers(0, len(res), size=n_views)
    out = []
    for v in range(n_views):
        W, H = res[int(picks[v])]
        spec = SceneSpec(n=int(counts[v]), s=4.0, z_lo=2.0, z_hi=20.0, width=W, height=H,
                         channels=channels, feat_dist="normal", opacity_range=(0.05, 0.95),
                         with_grad=True, seed=seed)
        out.append((spec, ring_camera(v, n_views, W, H)))
    return out


def multi_view_scenes(n_views: int = 8, seed: int = 0, **kw):
    """The scenes of the multi-view batch (see multi_view_specs)."""
    surfaces = draw_surfaces(np.random.default_rng(seed), 4.0, 2.0, 20.0)
    return [make_scene(spec, camera=cam, rng=np.random.default_rng([seed, v]), surfaces=surfaces)
            for v, (spec, cam) in enumerate(multi_view_specs(n_views, seed, **kw))]

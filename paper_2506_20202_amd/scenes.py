"""Seeded synthetic inputs: Gaussian scenes, cameras and clipping planes.

This module is the only code shared by the HIP path and the FP64 oracle.  It
draws inputs and nothing else: no projection, classification, weighting or
compositing happens here.  All sampling is done in float64 with
``numpy.random.default_rng(seed)`` and rounded once to float32, which is the
precision the renderer's inputs have.  Activations (``exp`` for scales, the
logistic function for opacities) are applied here because the renderer takes
linear standard deviations and post-activation opacity densities.

Workloads (stand-ins for the paper's trained scenes, which are not available):
  * ``tiny``       1,000 Gaussians, 128x128, SH degree 0 (the general-scene
                   shape of the method, small enough for the oracle);
  * ``general``    1,000,000 Gaussians in 64 anisotropic clusters, SH degree 3,
                   16 orbit views at 1920x1080, plane swept over 16 offsets
                   (stands in for the Mip-NeRF360 scenes of Sec. 4.1 / Table 1);
  * ``strands``    100,000 random-walk strands x 32 segments (3.2M Gaussians,
                   40:1:1 anisotropy), 8 views at 1024x1024 (stands in for the
                   hair scene of Sec. 4.1 / Table 1);
  * ``multilayer`` nested ellipsoidal shells with per-layer opacity (stands in
                   for the anatomical layered fields of Sec. 4.1);
  * ``diff``       500,000 general-scene Gaussians, 8 views at 800x800, one
                   plane per view, for the differentiable path.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

# Label values written by the classifier (Sec. 3.2): the same numbers are used
# by every consumer of labels.
INVISIBLE, VISIBLE, CUTOFF = 0, 1, 2


@dataclasses.dataclass
class Scene:
    """Gaussians in structure-of-arrays float32 layout.

    mean  [3][n]  centre mu (world units)
    scale [3][n]  per-axis standard deviation sigma (linear, not log)
    quat  [4][n]  rotation quaternion (w, x, y, z); need not be unit length
    opacity [n]   opacity density delta in (0, 1)
    sh    [(D+1)^2][3][n] real spherical-harmonic colour coefficients
    """

    mean: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.mean[:, idx]), np.ascontiguousarray(self.scale[:, idx]),
                     np.ascontiguousarray(self.quat[:, idx]), np.ascontiguousarray(self.opacity[idx]),
                     np.ascontiguousarray(self.sh[:, :, idx]), self.sh_degree)

    def arrays(self):
        return self.mean, self.scale, self.quat, self.opacity, self.sh


@dataclasses.dataclass
class Camera:
    """Pinhole camera: x right, y down, z forward.

    world_to_cam is the 3x4 matrix [R_c | t_c] (float32, row-major); a world
    point x maps to R_c x + t_c.  Pixel (i, j) has its centre at image
    coordinate (i, j) = (fx * x/z + cx, fy * y/z + cy).
    """

    world_to_cam: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2

    @property
    def tiles(self) -> Tuple[int, int]:
        return (self.width + 15) // 16, (self.height + 15) // 16


MAX_PLANES = 8


@dataclasses.dataclass
class Plane:
    """Clipping plane n.x + d = 0; the half-space n points into is visible.
    ``extra`` holds further planes (n, d): the visible region is then the
    intersection of all the half-spaces (a box is six of them)."""

    n: np.ndarray
    d: float
    enabled: bool = True
    extra: tuple = ()

    def as_array(self) -> np.ndarray:
        return np.array([self.n[0], self.n[1], self.n[2], self.d], dtype=np.float32)

    @property
    def count(self) -> int:
        return 1 + len(self.extra)

    def planes_array(self) -> np.ndarray:
        """[count][4] float32 rows (n.x, n.y, n.z, d), this plane first."""
        rows = [self.as_array()] + [np.array([n[0], n[1], n[2], d], dtype=np.float32) for n, d in self.extra]
        return np.ascontiguousarray(np.stack(rows))


def box_region(lo, hi, enabled=True) -> Plane:
    """The axis-aligned box lo <= x <= hi as six half-spaces."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    rows = []
    for a in range(3):
        e = np.zeros(3)
        e[a] = 1.0
        rows.append((_f32(e), float(np.float32(-lo[a]))))
        rows.append((_f32(-e), float(np.float32(hi[a]))))
    return Plane(rows[0][0], rows[0][1], enabled, tuple(rows[1:]))


def region(planes, enabled=True) -> Plane:
    """Intersection of the half-spaces of the given planes [(n, d), ...]."""
    rows = [(_f32(n), float(np.float32(d))) for n, d in planes]
    if not 1 <= len(rows) <= MAX_PLANES:
        raise ValueError(f"a region has 1 to {MAX_PLANES} planes")
    return Plane(rows[0][0], rows[0][1], enabled, tuple(rows[1:]))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _logistic(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _unit_vectors(rng, n):
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def _random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def _quat_from_frames(cols: np.ndarray) -> np.ndarray:
    """Quaternions (w,x,y,z) [4][n] of rotation matrices given as [n][3][3]
    (columns are the local axes).  Input synthesis only."""
    m = cols
    n = m.shape[0]
    q = np.zeros((n, 4))
    tr = m[:, 0, 0] + m[:, 1, 1] + m[:, 2, 2]
    cands = np.stack([tr, m[:, 0, 0], m[:, 1, 1], m[:, 2, 2]], axis=1)
    pick = np.argmax(cands, axis=1)
    for k in range(4):
        s = pick == k
        if not np.any(s):
            continue
        mm = m[s]
        if k == 0:
            r = np.sqrt(1.0 + tr[s]) * 2
            q[s] = np.stack([0.25 * r, (mm[:, 2, 1] - mm[:, 1, 2]) / r, (mm[:, 0, 2] - mm[:, 2, 0]) / r,
                             (mm[:, 1, 0] - mm[:, 0, 1]) / r], 1)
        elif k == 1:
            r = np.sqrt(1.0 + mm[:, 0, 0] - mm[:, 1, 1] - mm[:, 2, 2]) * 2
            q[s] = np.stack([(mm[:, 2, 1] - mm[:, 1, 2]) / r, 0.25 * r, (mm[:, 0, 1] + mm[:, 1, 0]) / r,
                             (mm[:, 0, 2] + mm[:, 2, 0]) / r], 1)
        elif k == 2:
            r = np.sqrt(1.0 + mm[:, 1, 1] - mm[:, 0, 0] - mm[:, 2, 2]) * 2
            q[s] = np.stack([(mm[:, 0, 2] - mm[:, 2, 0]) / r, (mm[:, 0, 1] + mm[:, 1, 0]) / r, 0.25 * r,
                             (mm[:, 1, 2] + mm[:, 2, 1]) / r], 1)
        else:
            r = np.sqrt(1.0 + mm[:, 2, 2] - mm[:, 0, 0] - mm[:, 1, 1]) * 2
            q[s] = np.stack([(mm[:, 1, 0] - mm[:, 0, 1]) / r, (mm[:, 0, 2] + mm[:, 2, 0]) / r,
                             (mm[:, 1, 2] + mm[:, 2, 1]) / r, 0.25 * r], 1)
    return q.T


def look_at(eye, target, up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """World-to-camera [R_c | t_c] (x right, y down, z forward) for a camera at
    ``eye`` looking at ``target`` with world ``up`` appearing upward."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    right = np.cross(f, np.asarray(up, np.float64))
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    rc = np.stack([right, down, f])
    tc = -rc @ eye
    return np.concatenate([rc, tc[:, None]], axis=1)


def pinhole(eye, target, width, height, vfov_deg, up=(0.0, 1.0, 0.0), near=0.2) -> Camera:
    """Camera with vertical field of view ``vfov_deg``; fx = fy = (H/2)/tan(fov/2),
    principal point at the image centre ((W-1)/2, (H-1)/2)."""
    f = (height / 2.0) / math.tan(math.radians(vfov_deg) / 2.0)
    return Camera(_f32(look_at(eye, target, up)), float(np.float32(f)), float(np.float32(f)),
                  float(np.float32((width - 1) / 2.0)), float(np.float32((height - 1) / 2.0)),
                  int(width), int(height), near)


def orbit_eye(radius, elevation_deg, azimuth_deg):
    el, az = math.radians(elevation_deg), math.radians(azimuth_deg)
    return np.array([radius * math.cos(el) * math.cos(az), radius * math.sin(el),
                     radius * math.cos(el) * math.sin(az)])


# ---------------------------------------------------------------- scenes ----

def tiny_scene(seed: int = 0, n: int = 1000) -> Scene:
    """Means U[-1,1]^3, log-scales N(-3, 0.5), uniform random rotations,
    opacity logistic(N(0,1)), RGB U[0,1] stored as the degree-0 SH coefficient
    (rgb - 0.5) / Y00 with Y00 = 1/(2 sqrt(pi))."""
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-1.0, 1.0, (3, n))
    scale = np.exp(rng.normal(-3.0, 0.5, (3, n)))
    quat = _unit_quats(rng, n)
    opacity = _logistic(rng.normal(0.0, 1.0, n))
    rgb = rng.uniform(0.0, 1.0, (3, n))
    y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    sh = ((rgb - 0.5) / y00)[None]
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(opacity), _f32(sh), 0)


def general_scene(seed: int = 1, n: int = 1_000_000, sh_degree: int = 3, clusters: int = 64) -> Scene:
    """Mixture of ``clusters`` anisotropic Gaussian clusters: centres U[-4,4]^3,
    per-axis std exp(U[ln 0.2, ln 1.0]) under a random rotation, equal weights,
    samples outside [-5,5]^3 redrawn.  log-scale N(-4, 0.8), opacity
    logistic(N(0, 1.5)), all SH coefficients N(0, 0.3)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-4.0, 4.0, (clusters, 3))
    stds = np.exp(rng.uniform(math.log(0.2), math.log(1.0), (clusters, 3)))
    rots = np.stack([_random_rotation(rng) for _ in range(clusters)])
    which = rng.integers(0, clusters, n)
    mean = np.empty((n, 3))
    todo = np.arange(n)
    while todo.size:
        c = which[todo]
        z = rng.standard_normal((todo.size, 3)) * stds[c]
        p = centres[c] + np.einsum("nij,nj->ni", rots[c], z)
        ok = np.all(np.abs(p) <= 5.0, axis=1)
        mean[todo[ok]] = p[ok]
        todo = todo[~ok]
    scale = np.exp(rng.normal(-4.0, 0.8, (3, n)))
    quat = _unit_quats(rng, n)
    opacity = _logistic(rng.normal(0.0, 1.5, n))
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.3, (k, 3, n))
    return Scene(_f32(mean.T), _f32(scale), _f32(quat), _f32(opacity), _f32(sh), sh_degree)


def strand_scene(seed: int = 2, strands: int = 100_000, segments: int = 32) -> Scene:
    """Random-walk strands rooted area-uniformly on the unit-sphere cap within
    60 degrees of +y.  The first tangent is the outward normal; each step turns
    it by N(0, 0.2 rad) about a random perpendicular axis and advances 0.02.
    One Gaussian per segment at its midpoint, major axis along the segment,
    random roll, scales (0.01, 2.5e-4, 2.5e-4), opacity logistic(N(1, 0.5)),
    SH degree 1 with coefficients N(0, 0.3)."""
    rng = np.random.default_rng(seed)
    cos_t = rng.uniform(0.5, 1.0, strands)
    phi = rng.uniform(0.0, 2 * math.pi, strands)
    sin_t = np.sqrt(1 - cos_t ** 2)
    p = np.stack([sin_t * np.cos(phi), cos_t, sin_t * np.sin(phi)], 1)
    t = p.copy()
    means, frames = [], []
    for _ in range(segments):
        a = rng.standard_normal((strands, 3))
        a -= np.sum(a * t, 1, keepdims=True) * t
        a /= np.linalg.norm(a, axis=1, keepdims=True)
        ang = rng.normal(0.0, 0.2, strands)[:, None]
        t = t * np.cos(ang) + np.cross(a, t) * np.sin(ang)
        t /= np.linalg.norm(t, axis=1, keepdims=True)
        q = p + 0.02 * t
        means.append(0.5 * (p + q))
        u = rng.standard_normal((strands, 3))
        u -= np.sum(u * t, 1, keepdims=True) * t
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        frames.append(np.stack([t, u, np.cross(t, u)], axis=2))
        p = q
    mean = np.concatenate(means, 0)
    quat = _quat_from_frames(np.concatenate(frames, 0))
    n = mean.shape[0]
    scale = np.tile(np.array([[0.01], [2.5e-4], [2.5e-4]]), (1, n))
    opacity = _logistic(rng.normal(1.0, 0.5, n))
    sh = rng.normal(0.0, 0.3, (4, 3, n))
    return Scene(_f32(mean.T), _f32(scale), _f32(quat), _f32(opacity), _f32(sh), 1)


def multilayer_scene(seed: int = 3, per_shell: int = 200_000, sh_degree: int = 0,
                     radii=(1.0, 1.25, 1.5, 1.75, 2.0), axes=(1.0, 0.8, 0.6),
                     layer_opacity=(0.95, 0.8, 0.6, 0.4, 0.2)) -> Scene:
    """Nested ellipsoidal shells (radius r times semi-axes ``axes``).  Gaussians
    lie on the shell with their short axis along the surface normal: tangential
    sigma 0.7 sqrt(area/count) exp(N(0, 0.2)), normal sigma one tenth of it.
    ``layer_opacity`` is listed inner to outer (outer layers are the most
    transparent).  SH coefficients N(0, 0.3)."""
    rng = np.random.default_rng(seed)
    ax = np.asarray(axes, np.float64)
    means, frames, scales, ops = [], [], [], []
    for li, r in enumerate(radii):
        u = _unit_vectors(rng, per_shell)
        semi = r * ax
        x = u * semi
        nrm = x / semi ** 2
        nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
        a = rng.standard_normal((per_shell, 3))
        a -= np.sum(a * nrm, 1, keepdims=True) * nrm
        a /= np.linalg.norm(a, axis=1, keepdims=True)
        b = np.cross(nrm, a)
        frames.append(np.stack([a, b, nrm], axis=2))
        p = 1.6075
        area = 4 * math.pi * (((semi[0] * semi[1]) ** p + (semi[0] * semi[2]) ** p + (semi[1] * semi[2]) ** p) / 3) ** (1 / p)
        st = 0.7 * math.sqrt(area / per_shell) * np.exp(rng.normal(0.0, 0.2, per_shell))
        scales.append(np.stack([st, st, 0.1 * st], 0))
        means.append(x)
        ops.append(np.full(per_shell, layer_opacity[li]))
    mean = np.concatenate(means, 0)
    quat = _quat_from_frames(np.concatenate(frames, 0))
    scale = np.concatenate(scales, 1)
    opacity = np.concatenate(ops)
    n = mean.shape[0]
    sh = rng.normal(0.0, 0.3, ((sh_degree + 1) ** 2, 3, n))
    return Scene(_f32(mean.T), _f32(scale), _f32(quat), _f32(opacity), _f32(sh), sh_degree)


# ------------------------------------------------------- cameras / planes ----

def tiny_camera(width: int = 128, height: int = 128) -> Camera:
    return pinhole((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), width, height, 60.0)


def tiny_plane(seed: int = 0) -> Plane:
    rng = np.random.default_rng(10_000 + seed)
    n = _unit_vectors(rng, 1)[0]
    return Plane(_f32(n), 0.0, True)


def general_views(count: int = 16, width: int = 1920, height: int = 1080, radius: float = 15.0,
                  elevation: float = 15.0) -> List[Camera]:
    return [pinhole(orbit_eye(radius, elevation, 360.0 * k / count), (0.0, 0.0, 0.0), width, height, 50.0)
            for k in range(count)]


def plane_sweep(scene: Scene, normal, count: int = 16, eps: float = 1e-3) -> List[Plane]:
    """``count`` planes with fixed unit normal whose offsets run from fully in
    front of every Gaussian's 3*max(sigma) ball (first) to fully behind (last).
    Uses only the scene's extent along the normal, not the classifier."""
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    proj = n @ scene.mean.astype(np.float64)
    rmax = 3.0 * float(scene.scale.max())
    lo, hi = proj.min() - rmax - eps, proj.max() + rmax + eps
    return [Plane(_f32(n), float(np.float32(-s)), True) for s in np.linspace(lo, hi, count)]


def general_plane_normal(seed: int = 1) -> np.ndarray:
    return _unit_vectors(np.random.default_rng(20_000 + seed), 1)[0]


def strand_views(count: int = 8, size: int = 1024) -> List[Camera]:
    return [pinhole(orbit_eye(4.0, 30.0, 360.0 * k / count), (0.0, 0.8, 0.0), size, size, 50.0)
            for k in range(count)]


def strand_planes(view: int, count: int = 8) -> List[Plane]:
    """Oblique planes, normal halfway between +y and the view's horizontal
    direction, through the strand shell at distances 1.0..1.6 from the origin."""
    az = math.radians(360.0 * view / count)
    n = np.array([math.cos(az), 1.0, math.sin(az)]) / math.sqrt(2.0)
    return [Plane(_f32(n), float(np.float32(-r)), True) for r in (1.0, 1.2, 1.4, 1.6)]


def diff_views(count: int = 8, size: int = 800, seed: int = 4, scene: Scene = None):
    """Eight 800x800 orbit views, each with a plane of random normal whose
    offset lies in the middle half of the scene's extent along that normal."""
    rng = np.random.default_rng(30_000 + seed)
    cams = [pinhole(orbit_eye(15.0, 15.0, 360.0 * k / count), (0.0, 0.0, 0.0), size, size, 50.0)
            for k in range(count)]
    planes = []
    for _ in range(count):
        n = _unit_vectors(rng, 1)[0]
        if scene is not None:
            proj = n @ scene.mean.astype(np.float64)
            q = rng.uniform(0.25, 0.75)
            off = float(np.quantile(proj, q))
        else:
            off = rng.uniform(-1.0, 1.0)
        planes.append(Plane(_f32(n), float(np.float32(-off)), True))
    return cams, planes


def perturbed(scene: Scene, seed: int = 4, mean_sigma: float = 0.01, logscale_sigma: float = 0.05) -> Scene:
    """Copy with means + N(0, 0.01) and log-scales + N(0, 0.05)."""
    rng = np.random.default_rng(40_000 + seed)
    mean = scene.mean.astype(np.float64) + rng.normal(0.0, mean_sigma, scene.mean.shape)
    scale = scene.scale.astype(np.float64) * np.exp(rng.normal(0.0, logscale_sigma, scene.scale.shape))
    return Scene(_f32(mean), _f32(scale), scene.quat.copy(), scene.opacity.copy(), scene.sh.copy(), scene.sh_degree)


def random_camera_on_sphere(rng, radius: float, width: int, height: int, vfov: float = 50.0) -> Camera:
    v = _unit_vectors(rng, 1)[0]
    up = (0.0, 1.0, 0.0) if abs(v[1]) < 0.95 else (1.0, 0.0, 0.0)
    return pinhole(radius * v, (0.0, 0.0, 0.0), width, height, vfov, up=up)


def random_plane_through(rng, scene: Scene) -> Plane:
    n = _unit_vectors(rng, 1)[0]
    proj = n @ scene.mean[:, :: max(1, scene.n // 20000)].astype(np.float64)
    off = rng.uniform(proj.min(), proj.max())
    return Plane(_f32(n), float(np.float32(-off)), True)


def small_scene(seed: int = 0, n: int = 12, spread: float = 0.35, logscale_mean: float = -2.0) -> Scene:
    """A handful of large anisotropic Gaussians near the origin (means
    U[-spread, spread]^3, log-scale N(logscale_mean, 0.3)), SH degree 0 with
    RGB U[0,1]; used where a brute-force checker must visit every pixel."""
    rng = np.random.default_rng(50_000 + seed)
    mean = rng.uniform(-spread, spread, (3, n))
    scale = np.exp(rng.normal(logscale_mean, 0.3, (3, n)))
    quat = _unit_quats(rng, n)
    opacity = _logistic(rng.normal(0.5, 1.0, n))
    rgb = rng.uniform(0.0, 1.0, (3, n))
    y00 = 1.0 / (2.0 * math.sqrt(math.pi))
    sh = ((rgb - 0.5) / y00)[None]
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(opacity), _f32(sh), 0)


def small_camera(size: int = 32) -> Camera:
    return pinhole((0.3, -0.4, -3.0), (0.0, 0.0, 0.0), size, size, 30.0)


def grad_scene(seed: int = 4, n: int = 200, sh_degree: int = 3) -> Scene:
    """General-scene statistics shrunk to a few hundred Gaussians in view of a
    64x64 camera (means N(0, 0.5^2), log-scale N(-2.5, 0.5), opacity
    logistic(N(0, 1.5)), SH coefficients N(0, 0.3)); used for gradient checks."""
    rng = np.random.default_rng(60_000 + seed)
    mean = rng.normal(0.0, 0.5, (3, n))
    scale = np.exp(rng.normal(-2.5, 0.5, (3, n)))
    quat = _unit_quats(rng, n)
    opacity = _logistic(rng.normal(0.0, 1.5, n))
    sh = rng.normal(0.0, 0.3, ((sh_degree + 1) ** 2, 3, n))
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(opacity), _f32(sh), sh_degree)


def grad_camera(size: int = 64) -> Camera:
    return pinhole((1.0, 0.8, -4.0), (0.0, 0.0, 0.0), size, size, 50.0)


def grad_plane(seed: int = 4) -> Plane:
    rng = np.random.default_rng(70_000 + seed)
    n = _unit_vectors(rng, 1)[0]
    return Plane(_f32(n), float(np.float32(rng.uniform(-0.1, 0.1))), True)


def concat(*parts: Scene) -> Scene:
    """One scene holding the Gaussians of ``parts`` in order (same SH degree)."""
    deg = parts[0].sh_degree
    assert all(p.sh_degree == deg for p in parts)
    return Scene(*(np.ascontiguousarray(np.concatenate([getattr(p, f) for p in parts], axis=-1))
                   for f in ("mean", "scale", "quat", "opacity", "sh")), deg)


def wide_gaussians(seed: int = 0, n: int = 6, sh_degree: int = 3, sigma=(0.4, 0.6),
                   opacity: float = 0.3) -> Scene:
    """A few large anisotropic Gaussians near the origin (per-axis sigma
    U[sigma], means N(0, 0.15^2)): at a grad_camera of 128 px or more their
    footprints span most of the image, over 32 tiles each."""
    rng = np.random.default_rng(80_000 + seed)
    mean = rng.normal(0.0, 0.15, (3, n))
    scale = rng.uniform(sigma[0], sigma[1], (3, n))
    quat = _unit_quats(rng, n)
    op = np.full(n, opacity)
    sh = rng.normal(0.0, 0.3, ((sh_degree + 1) ** 2, 3, n))
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(op), _f32(sh), sh_degree)


def faint_list_scene(seed: int = 0, n: int = 1500, opacity: float = 0.0058, sh_degree: int = 3,
                     spread: float = 0.1, sigma=(0.8, 1.2)) -> Scene:
    """``n`` large, faint Gaussians in a small cluster (means U[-spread,
    spread]^3, per-axis sigma U[sigma], opacity ``opacity``).  Seen by
    ``faint_camera`` every pixel is within a fraction of a sigma of every
    centre, so alpha stays within about 25 % of ``opacity``: each tile list
    holds all n Gaussians, every entry is composited, and no pixel terminates
    (the product of (1 - alpha) over the list stays above 1e-4)."""
    rng = np.random.default_rng(90_000 + seed)
    mean = rng.uniform(-spread, spread, (3, n))
    scale = rng.uniform(sigma[0], sigma[1], (3, n))
    quat = _unit_quats(rng, n)
    op = np.full(n, opacity)
    sh = rng.normal(0.0, 0.3, ((sh_degree + 1) ** 2, 3, n))
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(op), _f32(sh), sh_degree)


def faint_camera(size: int = 32) -> Camera:
    """A narrow (9 degree) view of the faint cluster from distance about 6.3."""
    return pinhole((1.5, 1.2, -6.0), (0.0, 0.0, 0.0), size, size, 9.0)


def inside_gaussian(cam: Camera, depth: float = 0.5, sigma=(0.3, 0.3, 0.3), opacity: float = 0.4,
                    sh_degree: int = 3, seed: int = 0) -> Scene:
    """One Gaussian centred ``depth`` in front of the camera on its optical
    axis: with 3 sigma > depth the camera lies inside its 3-sigma ellipsoid
    (the case where the near root of the ray-ellipsoid quadratic is behind the
    camera)."""
    rng = np.random.default_rng(95_000 + seed)
    wc = np.asarray(cam.world_to_cam, np.float64).reshape(3, 4)
    eye = -wc[:, :3].T @ wc[:, 3]
    fwd = wc[2, :3]
    mean = (eye + depth * fwd)[:, None]
    scale = np.asarray(sigma, np.float64)[:, None]
    quat = _unit_quats(rng, 1)
    sh = rng.normal(0.0, 0.3, ((sh_degree + 1) ** 2, 3, 1))
    return Scene(_f32(mean), _f32(scale), _f32(quat), _f32(np.array([opacity])), _f32(sh), sh_degree)


def plane_through(point, normal, enabled=True) -> Plane:
    """Plane with unit normal ``normal`` through ``point``."""
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    return Plane(_f32(n), float(np.float32(-float(n @ np.asarray(point, np.float64)))), enabled)

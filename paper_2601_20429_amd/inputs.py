"""Seeded synthetic inputs for the Gaussian ray tracer: scenes, cameras and rays.

This module is shared by the tests, the benchmark and the oracle-side checks. It holds
random draws and their packing only; none of the rendering arithmetic (ray generation
from a camera, ray/Gaussian intersection, alpha, colour, compositing) lives here.

The trained scenes of the paper's evaluation (Tanks&Temples, Mip-NeRF 360, Deep
Blending; Sec. V-A, Table "Summary of workloads") are not available, so seeded
synthetic scenes of the same scale stand in for them (0.1-3 M Gaussians against the
paper's 0.76-2.43 M).

Conventions (the parameterisation of a Gaussian, Sec. II-B):
  means  [N,3]  centre mu
  scales [N,3]  linear per-axis standard deviation s (Sigma = R diag(s)^2 R^T)
  quats  [N,4]  rotation quaternion (w, x, y, z); need not be normalised
  opac   [N]    opacity o in (0, 1)
  sh     [N,(L+1)^2,3] real spherical-harmonic colour coefficients, band-major,
         m = -l..l inside band l, RGB innermost
All arrays are float32 and C-contiguous.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Real SH band-0 basis value 1/(2 sqrt(pi)); used only to encode a plain RGB colour as
# a degree-0 coefficient (rgb = 0.5 + Y00 * sh0).
_Y00 = 0.5 / math.sqrt(math.pi)


@dataclasses.dataclass
class Scene:
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacities: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.means[idx]), np.ascontiguousarray(self.scales[idx]),
                     np.ascontiguousarray(self.quats[idx]), np.ascontiguousarray(self.opacities[idx]),
                     np.ascontiguousarray(self.sh[idx]), self.sh_degree)


@dataclasses.dataclass
class Camera:
    """Pinhole camera: eye, look-at target, up hint, vertical field of view, image size."""
    eye: tuple
    target: tuple
    up: tuple
    fov_y_deg: float
    width: int
    height: int

    @property
    def n_rays(self) -> int:
        return self.width * self.height


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _random_rotations(rng, n):
    """Random 3x3 rotations from the QR factorisation of Gaussian matrices."""
    g = rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diagonal(r, axis1=1, axis2=2))
    s[s == 0] = 1.0
    q = q * s[:, None, :]
    det = np.linalg.det(q)
    q[det < 0, :, 0] *= -1.0
    return q


def _sh_coeffs(rng, n, degree, dc_std, rest_std):
    k = (degree + 1) ** 2
    sh = np.empty((n, k, 3))
    sh[:, 0, :] = rng.normal(0.0, dc_std, (n, 3))
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, rest_std, (n, k - 1, 3))
    return sh


def small_scene(seed: int = 1, n: int = 1000) -> Scene:
    """Plain-method scene: 8 isotropic clusters (sigma 0.2, centres in [-1,1]^3), per-axis
    scale exp(N(-3, 0.5)), uniform random rotation, opacity sigmoid(N(0, 1.5)), RGB DC
    colour N(0.5, 0.2) clipped to [0, 1], SH degree 0."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-1.0, 1.0, (8, 3))
    which = rng.integers(0, 8, n)
    means = centres[which] + rng.normal(0.0, 0.2, (n, 3))
    scales = np.exp(rng.normal(-3.0, 0.5, (n, 3)))
    quats = _unit_quats(rng, n)
    opac = _sigmoid(rng.normal(0.0, 1.5, n))
    rgb = np.clip(rng.normal(0.5, 0.2, (n, 3)), 0.0, 1.0)
    sh = ((rgb - 0.5) / _Y00)[:, None, :]
    return Scene(_f32(means), _f32(scales), _f32(quats), _f32(opac), _f32(sh), 0)


def cluster_scene(seed: int, n: int, sh_degree: int = 3) -> Scene:
    """Scene-scale synthetic scene: 90% of the Gaussians from 32 anisotropic clusters
    (centre U[-1,1]^3, covariance R diag(sigma^2) R^T with sigma ~ U(0.05, 0.35) per axis),
    10% uniform in [-1.5, 1.5]^3; per-axis scale exp(N(-4.5, 0.8)); opacity
    sigmoid(N(0, 1.5)); SH degree 3 with DC ~ N(0, 0.5) and higher bands ~ N(0, 0.1)."""
    rng = np.random.default_rng(seed)
    n_cl = int(round(0.9 * n))
    n_bg = n - n_cl
    centres = rng.uniform(-1.0, 1.0, (32, 3))
    rot = _random_rotations(rng, 32)
    sig = rng.uniform(0.05, 0.35, (32, 3))
    which = rng.integers(0, 32, n_cl)
    z = rng.standard_normal((n_cl, 3)) * sig[which]
    pts = centres[which] + np.einsum("nij,nj->ni", rot[which], z)
    bg = rng.uniform(-1.5, 1.5, (n_bg, 3))
    means = np.concatenate([pts, bg], axis=0)
    means = means[rng.permutation(n)]
    scales = np.exp(rng.normal(-4.5, 0.8, (n, 3)))
    quats = _unit_quats(rng, n)
    opac = _sigmoid(rng.normal(0.0, 1.5, n))
    sh = _sh_coeffs(rng, n, sh_degree, 0.5, 0.1)
    return Scene(_f32(means), _f32(scales), _f32(quats), _f32(opac), _f32(sh), sh_degree)


def fd_scene(seed: int = 5, n: int = 500) -> Scene:
    """Small differentiable test scene: 8 isotropic clusters (sigma 0.2, centres in
    [-1,1]^3), per-axis scale exp(N(-2.5, 0.4)), uniform rotation, opacity
    sigmoid(N(0, 1.5)), SH degree 3 (DC ~ N(0, 0.5), higher bands ~ N(0, 0.1))."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-1.0, 1.0, (8, 3))
    which = rng.integers(0, 8, n)
    means = centres[which] + rng.normal(0.0, 0.2, (n, 3))
    scales = np.exp(rng.normal(-2.5, 0.4, (n, 3)))
    quats = _unit_quats(rng, n)
    opac = _sigmoid(rng.normal(0.0, 1.5, n))
    sh = _sh_coeffs(rng, n, 3, 0.5, 0.1)
    return Scene(_f32(means), _f32(scales), _f32(quats), _f32(opac), _f32(sh), 3)


def perturbed_means(scene: Scene, seed: int, std: float = 0.01) -> Scene:
    """Copy of `scene` with means + N(0, std^2) (target scene of the differentiation case)."""
    rng = np.random.default_rng(seed)
    means = scene.means.astype(np.float64) + rng.normal(0.0, std, scene.means.shape)
    return dataclasses.replace(scene, means=_f32(means))


def orbit_camera(width: int, height: int, eye=(0.0, -3.0, 0.0), fov_y_deg: float = 60.0) -> Camera:
    """Camera at `eye` looking at the origin with +z as the up hint."""
    return Camera(tuple(float(x) for x in eye), (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), float(fov_y_deg),
                  int(width), int(height))


def random_orbit_eye(rng, radius: float = 3.0):
    """Uniform point on the sphere of the given radius (avoiding the poles, where the +z up
    hint is parallel to the view direction)."""
    while True:
        v = rng.standard_normal(3)
        v /= np.linalg.norm(v)
        if abs(v[2]) < 0.98:
            return tuple(float(x) for x in radius * v)


def incoherent_rays(seed: int, count: int, box: float = 1.5):
    """Rays with origins uniform in [-box, box]^3 and directions uniform on the sphere.
    Returns float32 origins [count,3] and unit directions [count,3]."""
    rng = np.random.default_rng(seed)
    o = rng.uniform(-box, box, (count, 3))
    d = rng.standard_normal((count, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return _f32(o), _f32(d)


def ray_subsample(seed: int, total: int, count: int) -> np.ndarray:
    """Sorted, distinct ray indices drawn without replacement."""
    rng = np.random.default_rng(seed)
    count = min(count, total)
    return np.sort(rng.choice(total, size=count, replace=False)).astype(np.int64)


def secondary_objects(seed: int = 60) -> dict:
    """A glass sphere and a rectangular mirror at seeded random places in front of the
    orbit camera at (0, -3, 0) (the secondary-ray experiment places one of each in every
    scene). Sphere: centre uniform in [-0.8, 0.8] x [-1, 0] x [-0.5, 0.5], radius uniform
    in [0.35, 0.5], index 1.5. Mirror: centre uniform in [-1, 1] x [0, 0.8] x [-0.5, 0.5],
    normal (s * U(0.6, 1.4), -1, N(0, 0.3)) normalised with a random sign s (turned
    towards the camera and to one side, so that reflections run through the scene),
    half-axes 0.7 and 0.5 orthogonal to it. Returns {"sphere": (cx, cy, cz, r, ior),
    "mirror": (m, u, v) as 9 numbers, "eps": 1e-4} in float32-representable values."""
    rng = np.random.default_rng(seed)
    c = rng.uniform([-0.8, -1.0, -0.5], [0.8, 0.0, 0.5])
    r = rng.uniform(0.35, 0.5)
    m = rng.uniform([-1.0, 0.0, -0.5], [1.0, 0.8, 0.5])
    n = np.array([rng.choice([-1.0, 1.0]) * rng.uniform(0.6, 1.4), -1.0, rng.normal(0.0, 0.3)])
    n /= np.linalg.norm(n)
    a = np.cross(n, [0.0, 0.0, 1.0])
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    u, v = 0.7 * a, 0.5 * b
    f = lambda x: [float(np.float32(t)) for t in np.ravel(x)]
    return {"sphere": tuple(f(c) + f(r) + [1.5]), "mirror": tuple(f(m) + f(u) + f(v)), "eps": 1e-4}


# Named workloads. Sizes follow the plain-method case, the scene-scale cases, the
# differentiation case and the serving case.
PLAIN = dict(name="plain-1k-64x64-k4", seed=1, n=1000, width=64, height=64, k=4,
             alpha_min=1.0 / 255.0, T_min=1e-3)
SCENE100K = dict(name="scene-100k-800x800-k16", seed=2, n=100_000, width=800, height=800, k=16,
                 alpha_min=1.0 / 255.0, T_min=1e-3)
SCENE3M = dict(name="scene-3M-1920x1080+2Mincoherent-k16", seed=3, n=3_000_000, width=1920,
               height=1080, incoherent=2_000_000, incoherent_seed=33, k=16,
               alpha_min=1.0 / 255.0, T_min=1e-3)
DIFF200K = dict(name="diff-200k-512x512-k16", seed=4, n=200_000, width=512, height=512, k=16,
                target_seed=44, fd_seed=5, fd_n=500, fd_width=32, fd_height=32,
                alpha_min=1.0 / 255.0, T_min=1e-3)
SECONDARY = dict(name="scene-100k-800x800-k16+glass+mirror", seed=2, n=100_000, width=800, height=800, k=16,
                 objects_seed=60, alpha_min=1.0 / 255.0, T_min=1e-3)
SERVE = dict(name="serve-4scenes-poisson200", scene_seeds=(10, 11, 12, 13),
             scene_sizes=(100_000, 500_000, 1_000_000, 3_000_000), rate=200.0, arrival_seed=50,
             resolutions=((256, 256), (512, 512), (800, 800), (1920, 1080)), k=16,
             alpha_min=1.0 / 255.0, T_min=1e-3)


def make_workload_scene(cfg: dict) -> Scene:
    if cfg["n"] <= 1000 and cfg["seed"] == 1:
        return small_scene(cfg["seed"], cfg["n"])
    return cluster_scene(cfg["seed"], cfg["n"], 3)

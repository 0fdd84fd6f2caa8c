"""Seeded synthetic inputs: scenes, cameras and target images.

This module draws random numbers and builds camera poses; it holds none of
the rasterizer's arithmetic, so the HIP path and the FP64 oracle can both be
fed from it.  All arrays are numpy FP32 (the library's input precision).

The paper trains on Mip-NeRF360, Tanks&Temples and Deep Blending; none of
those are used here.  These generators stand in for them with the component
counts, resolutions and parameter distributions of the workloads below.

Workloads (sizes per view):
  small      10k components, SH degree 0, one 256x256 camera at (0, 0, 4)
  train      300k components, SH degree 3, one 1297x840 camera on a ring
  m1         1M components, SH degree 3, one 1920x1080 camera on a ring
  large      3M clustered components, nu log-uniform in [1, 150], 30% negative
  multiview  5M clustered components, 8 cameras 1600x1064 on a ring
"""
from __future__ import annotations

import math

import numpy as np

SEED_SCENE, SEED_CAMERA, SEED_TARGET, SEED_FD, SEED_SGHMC, SEED_ARRIVALS = 0, 1, 2, 3, 4, 5

# the degree-0 SH coefficient that maps to a colour in [0, 1] spans
# [-sqrt(pi), sqrt(pi)] (0.5 / Y00 = sqrt(pi))
_DC_HALF_RANGE = math.sqrt(math.pi)


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def make_scene(n: int, sh_degree: int = 0, seed: int = SEED_SCENE, layout: str = "uniform",
               neg_frac: float = 0.2, nu_mode: str = "exp", n_clusters: int = 200,
               scale_range=(0.005, 0.05)) -> dict:
    """Random scene of n signed Student's t components (activated values).

    layout  "uniform": means ~ U[-1, 1]^3;  "clusters": means from a mixture
            of n_clusters anisotropic Gaussians (centres U[-1,1]^3, per-axis
            std log-uniform in [0.02, 0.3], random rotation, uniform choice).
    nu_mode "exp": nu = 1 + exp(U[-1, 4]);  "loguniform": nu log-uniform [1, 150].
    Opacity: (1 - neg_frac) of the components U(0.05, 0.95), the rest
    -U(0.05, 0.5).  Scales log-uniform in scale_range per axis.  SH: DC term
    gives a colour U(0, 1); higher coefficients N(0, 0.2).
    """
    rng = np.random.default_rng(seed)
    if layout == "uniform":
        means = rng.uniform(-1.0, 1.0, (n, 3))
    elif layout == "clusters":
        centres = rng.uniform(-1.0, 1.0, (n_clusters, 3))
        stds = np.exp(rng.uniform(math.log(0.02), math.log(0.3), (n_clusters, 3)))
        # random rotations: Q factor of a Gaussian matrix, sign-fixed to det +1
        Q, Rr = np.linalg.qr(rng.standard_normal((n_clusters, 3, 3)))
        Q = Q * np.sign(np.diagonal(Rr, axis1=1, axis2=2))[:, None, :]
        Q[np.linalg.det(Q) < 0, :, 0] *= -1.0
        R = Q
        choice = rng.integers(0, n_clusters, n)
        local = rng.standard_normal((n, 3)) * stds[choice]
        means = centres[choice] + np.einsum("nij,nj->ni", R[choice], local)
    else:
        raise ValueError(layout)
    lo, hi = scale_range
    scales = np.exp(rng.uniform(math.log(lo), math.log(hi), (n, 3)))
    quats = _unit_quats(rng, n)
    if nu_mode == "exp":
        nu = 1.0 + np.exp(rng.uniform(-1.0, 4.0, n))
    elif nu_mode == "loguniform":
        nu = np.exp(rng.uniform(0.0, math.log(150.0), n))
    else:
        raise ValueError(nu_mode)
    neg = rng.uniform(0.0, 1.0, n) < neg_frac
    opacity = np.where(neg, -rng.uniform(0.05, 0.5, n), rng.uniform(0.05, 0.95, n))
    K = (sh_degree + 1) ** 2
    sh = np.zeros((n, K, 3))
    sh[:, 0, :] = rng.uniform(-_DC_HALF_RANGE, _DC_HALF_RANGE, (n, 3))
    if K > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.2, (n, K - 1, 3))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(means=f32(means), scales=f32(scales), quats=f32(quats), nu=f32(nu),
                opacity=f32(opacity), sh=f32(sh), sh_degree=int(sh_degree))


def lookat_camera(eye, target, width: int, height: int, fov_x_deg: float = 60.0,
                  up=(0.0, 1.0, 0.0)) -> dict:
    """Pinhole camera, OpenCV axes (x right, y down, z forward), principal
    point at the image centre, fx = fy from the horizontal field of view."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f], 0)
    t = -R @ eye
    viewmat = np.concatenate([R, t[:, None]], 1).astype(np.float32)
    fx = width / (2.0 * math.tan(math.radians(fov_x_deg) / 2.0))
    return dict(viewmat=viewmat, fx=float(np.float32(fx)), fy=float(np.float32(fx)),
                cx=float(np.float32(width / 2.0)), cy=float(np.float32(height / 2.0)),
                width=int(width), height=int(height))


def ring_camera(width: int, height: int, radius: float = 4.0, angle: float | None = None,
                seed: int = SEED_CAMERA) -> dict:
    """Camera on the xz-ring of the given radius looking at the origin."""
    if angle is None:
        angle = np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi)
    eye = (radius * math.sin(angle), 0.0, radius * math.cos(angle))
    return lookat_camera(eye, (0.0, 0.0, 0.0), width, height)


def ring_cameras(n_views: int, width: int, height: int, radius: float = 4.0,
                 seed: int = SEED_CAMERA) -> list:
    a0 = np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi)
    return [ring_camera(width, height, radius, a0 + 2.0 * math.pi * v / n_views) for v in range(n_views)]


def sphere_camera(rng, width: int, height: int, rmin: float = 3.0, rmax: float = 5.0) -> dict:
    """Direction uniform on the sphere (redrawn if |y| > 0.99), radius U[rmin, rmax]."""
    while True:
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        if abs(d[1]) <= 0.99:
            break
    eye = d * rng.uniform(rmin, rmax)
    return lookat_camera(eye, (0.0, 0.0, 0.0), width, height)


def smooth_target(width: int, height: int, seed: int = SEED_TARGET) -> np.ndarray:
    """Random smooth noise image [H, W, 3]: U(0, 1) on a coarse grid with
    32-pixel spacing, bilinearly upsampled."""
    rng = np.random.default_rng(seed)
    gh, gw = height // 32 + 2, width // 32 + 2
    grid = rng.uniform(0.0, 1.0, (gh, gw, 3))
    ys = (np.arange(height) + 0.5) / 32.0
    xs = (np.arange(width) + 0.5) / 32.0
    y0 = np.floor(ys).astype(int)
    x0 = np.floor(xs).astype(int)
    fy = (ys - y0)[:, None, None]
    fx = (xs - x0)[None, :, None]
    g00 = grid[y0][:, x0]
    g01 = grid[y0][:, x0 + 1]
    g10 = grid[y0 + 1][:, x0]
    g11 = grid[y0 + 1][:, x0 + 1]
    img = (1 - fy) * ((1 - fx) * g00 + fx * g01) + fy * ((1 - fx) * g10 + fx * g11)
    return np.ascontiguousarray(img, dtype=np.float32)


def workload(name: str):
    """(scene, cameras) of a named workload."""
    if name == "small":
        return make_scene(10_000, 0), [lookat_camera((0.0, 0.0, 4.0), (0.0, 0.0, 0.0), 256, 256)]
    if name == "train":
        return make_scene(300_000, 3), [ring_camera(1297, 840)]
    if name == "m1":
        return make_scene(1_000_000, 3), [ring_camera(1920, 1080)]
    if name == "large":
        return (make_scene(3_000_000, 3, layout="clusters", neg_frac=0.3, nu_mode="loguniform"),
                [ring_camera(1920, 1080)])
    if name == "multiview":
        return (make_scene(5_000_000, 3, layout="clusters", neg_frac=0.3, nu_mode="loguniform"),
                ring_cameras(8, 1600, 1064))
    raise KeyError(name)

"""Seeded synthetic inputs: Gaussian scenes, cameras, target images and change sets.

This module is the only code shared by the CPU reference (``oracle/``) and the GPU
library (``paper_2506_21117_amd``).  It draws random numbers and builds camera poses;
it computes nothing the renderer computes (no projection, no colour, no compositing).

Conventions of the data it produces
-----------------------------------
* Gaussian parameters are raw (pre-activation) float32 arrays in component-major
  (SoA) layout, exactly the layout the C-ABI takes:
  ``means[3][N]``, ``log_scales[3][N]``, ``quats[4][N]`` (w, x, y, z, not normalised),
  ``opacity_logit[N]``, ``sh[K][3][N]`` with ``K = (D+1)**2`` spherical-harmonic
  coefficients per colour channel.
* Cameras use the OpenCV frame (x right, y down, z forward); ``R`` maps world to
  camera (row-major 3x3) and ``t`` is the world-to-camera translation, so a world
  point ``x`` sits at ``R @ x + t`` in camera space.  Every camera value is float32.

The workloads follow the paper's setting (Sec. 3 problem statement: an existing
reconstruction, new posed images, and a 3D change set O^t; Supp. "History Recovery":
the static Gaussians are stored first and the changed ones last).  The paper's datasets
are not available, so these generators stand in for them; the recipes are listed in
the design notes of the repository.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

# Distribution width for the degree-0 colour coefficient so that the DC colour term
# covers [0, 1] (the renderer adds 0.5 to the SH sum); 1/0.28209479177387814.
_DC_SPAN = 3.5449077018110318


@dataclass
class Camera:
    R: np.ndarray          # float32 [3, 3], world -> camera rotation
    t: np.ndarray          # float32 [3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int

    def __post_init__(self):
        self.R = np.ascontiguousarray(self.R, dtype=np.float32).reshape(3, 3)
        self.t = np.ascontiguousarray(self.t, dtype=np.float32).reshape(3)
        self.fx = float(np.float32(self.fx))
        self.fy = float(np.float32(self.fy))
        self.cx = float(np.float32(self.cx))
        self.cy = float(np.float32(self.cy))
        self.width = int(self.width)
        self.height = int(self.height)


@dataclass
class Scene:
    means: np.ndarray          # [3, N]
    log_scales: np.ndarray     # [3, N]
    quats: np.ndarray          # [4, N]
    opacity_logit: np.ndarray  # [N]
    sh: np.ndarray             # [K, 3, N]
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def __post_init__(self):
        for name in ("means", "log_scales", "quats", "opacity_logit", "sh"):
            setattr(self, name, np.ascontiguousarray(getattr(self, name), dtype=np.float32))
        n = self.means.shape[1]
        k = (self.sh_degree + 1) ** 2
        assert self.means.shape == (3, n)
        assert self.log_scales.shape == (3, n)
        assert self.quats.shape == (4, n)
        assert self.opacity_logit.shape == (n,)
        assert self.sh.shape == (k, 3, n), (self.sh.shape, k, n)

    def take(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[:, idx], self.log_scales[:, idx], self.quats[:, idx],
                     self.opacity_logit[idx], self.sh[:, :, idx], self.sh_degree)

    def copy(self) -> "Scene":
        return Scene(self.means.copy(), self.log_scales.copy(), self.quats.copy(),
                     self.opacity_logit.copy(), self.sh.copy(), self.sh_degree)

    def param_arrays(self):
        return [self.means, self.log_scales, self.quats, self.opacity_logit, self.sh]


def concat(a: Scene, b: Scene) -> Scene:
    assert a.sh_degree == b.sh_degree
    return Scene(np.concatenate([a.means, b.means], 1),
                 np.concatenate([a.log_scales, b.log_scales], 1),
                 np.concatenate([a.quats, b.quats], 1),
                 np.concatenate([a.opacity_logit, b.opacity_logit]),
                 np.concatenate([a.sh, b.sh], 2), a.sh_degree)


# --------------------------------------------------------------------------- cameras
def look_at(center, target=(0.0, 0.0, 0.0), down=(0.0, 1.0, 0.0), *, width, height,
            fx, fy=None, cx=None, cy=None) -> Camera:
    """Pinhole camera at ``center`` looking at ``target`` (OpenCV axes, image y along
    the world ``down`` direction)."""
    c = np.asarray(center, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - c
    f /= np.linalg.norm(f)
    x = np.cross(np.asarray(down, dtype=np.float64), f)
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    R = np.stack([x, y, f]).astype(np.float32)
    t = (-(R.astype(np.float64) @ c)).astype(np.float32)
    fy = fx if fy is None else fy
    cx = width / 2.0 if cx is None else cx
    cy = height / 2.0 if cy is None else cy
    return Camera(R, t, fx, fy, cx, cy, width, height)


def ring_cameras(n_views, radius, *, width, height, fx, fy=None, phase=0.0):
    cams = []
    for k in range(n_views):
        th = phase + 2.0 * math.pi * k / n_views
        cams.append(look_at((radius * math.sin(th), 0.0, -radius * math.cos(th)),
                            width=width, height=height, fx=fx, fy=fy))
    return cams


def sphere_camera(rng, radius, *, width, height, fx):
    while True:
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        if abs(d[1]) < 0.95:          # keep the look direction away from the up axis
            return look_at(radius * d, width=width, height=height, fx=fx)


# --------------------------------------------------------------------------- scenes
def _random_quats(rng, n):
    return rng.normal(size=(4, n)).astype(np.float32)


def uniform_cube_scene(rng, n, *, sh_degree=0, extent=1.0, log_scale_mean=-3.0,
                       log_scale_sd=0.5, sh_rest_sd=0.3) -> Scene:
    """Means uniform in [-extent, extent]^3, per-axis log-scales N(mean, sd), random
    quaternions, opacity logits N(0, 1), DC colour uniform in [0, 1] and higher SH
    bands N(0, sh_rest_sd)."""
    means = rng.uniform(-extent, extent, size=(3, n)).astype(np.float32)
    log_scales = rng.normal(log_scale_mean, log_scale_sd, size=(3, n)).astype(np.float32)
    quats = _random_quats(rng, n)
    opacity_logit = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    k = (sh_degree + 1) ** 2
    sh = np.empty((k, 3, n), dtype=np.float32)
    sh[0] = ((rng.uniform(0.0, 1.0, size=(3, n)) - 0.5) * _DC_SPAN).astype(np.float32)
    if k > 1:
        sh[1:] = rng.normal(0.0, sh_rest_sd, size=(k - 1, 3, n)).astype(np.float32)
    return Scene(means, log_scales, quats, opacity_logit, sh, sh_degree)


def gaussian_cloud_scene(rng, n, *, sh_degree=3, sigma=1.5, log_scale_mean=-4.0,
                         log_scale_sd=0.7, sh_sd=0.3) -> Scene:
    """Means from N(0, sigma^2 I); every SH coefficient N(0, sh_sd)."""
    means = rng.normal(0.0, sigma, size=(3, n)).astype(np.float32)
    log_scales = rng.normal(log_scale_mean, log_scale_sd, size=(3, n)).astype(np.float32)
    quats = _random_quats(rng, n)
    opacity_logit = rng.normal(0.0, 1.0, size=n).astype(np.float32)
    k = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, sh_sd, size=(k, 3, n)).astype(np.float32)
    return Scene(means, log_scales, quats, opacity_logit, sh, sh_degree)


def reinit_like_new_points(rng, scene: Scene, idx, *, log_scale_mean=-4.26, log_scale_sd=0.24,
                           opacity=0.1) -> Scene:
    """Re-initialise the Gaussians ``idx`` the way freshly sampled points start
    (Sec. 3.2, "Gaussian Sampling for New Objects": standard SfM-style initialisation):
    positions uniform inside the bounding sphere of the old ones, isotropic small
    scales, low opacity, random colour, zero higher SH bands."""
    idx = np.asarray(idx)
    out = scene.copy()
    m = len(idx)
    if m == 0:
        return out
    pts = scene.means[:, idx].astype(np.float64)
    center = pts.mean(axis=1, keepdims=True)
    radius = float(np.max(np.linalg.norm(pts - center, axis=0))) if m > 1 else 0.1
    d = rng.normal(size=(3, m))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    r = radius * rng.uniform(0.0, 1.0, size=m) ** (1.0 / 3.0)
    out.means[:, idx] = (center + d * r).astype(np.float32)
    ls = rng.normal(log_scale_mean, log_scale_sd, size=m).astype(np.float32)
    out.log_scales[:, idx] = np.broadcast_to(ls, (3, m))
    q = np.zeros((4, m), dtype=np.float32)
    q[0] = 1.0
    out.quats[:, idx] = q
    out.opacity_logit[idx] = np.float32(math.log(opacity / (1.0 - opacity)))
    out.sh[:, :, idx] = 0.0
    out.sh[0, :, idx] = ((rng.uniform(0.0, 1.0, size=(m, 3)) - 0.5) * _DC_SPAN).astype(np.float32)
    return out


def static_first(scene: Scene, active_mask):
    """Reorder so the unchanged Gaussians come first and the change set last
    (Supp. "History Recovery": the first #static Gaussians of G^t are G^{t-1}
    without O^t).  Returns (scene, a0, perm) with the change set at [a0, N)."""
    active_mask = np.asarray(active_mask, dtype=bool)
    perm = np.concatenate([np.nonzero(~active_mask)[0], np.nonzero(active_mask)[0]])
    return scene.take(perm), int((~active_mask).sum()), perm


def random_target(rng, n_views, height, width):
    return rng.uniform(0.0, 1.0, size=(n_views, 3, height, width)).astype(np.float32)


# --------------------------------------------------------------------------- workloads
@dataclass
class Workload:
    name: str
    scene: Scene
    cameras: list
    active_begin: int = 0                 # change set O^t = [active_begin, N)
    targets: np.ndarray | None = None     # [V, 3, H, W] float32 or None
    scene_gt: Scene | None = None
    extra: dict = field(default_factory=dict)


def tiny(seed=1, n=2000, width=128, height=128, sh_degree=0) -> Workload:
    """2 000 Gaussians uniform in [-1, 1]^3, camera at distance 4, one 128x128 view
    with fx = fy = 128, uniform random target."""
    rng = np.random.default_rng(seed)
    sc = uniform_cube_scene(rng, n, sh_degree=sh_degree)
    cam = Camera(np.eye(3), (0.0, 0.0, 4.0), width, width, width / 2.0, height / 2.0, width, height)
    tgt = random_target(rng, 1, height, width)
    return Workload("tiny-2k-128px", sc, [cam], 0, tgt)


def full_scene(seed=2, n=200_000, n_views=8, res=800, fx=1100.0) -> Workload:
    """200k Gaussians from an N(0, 1.5^2 I) cloud, SH degree 3, 8 ring views of
    800x800 at radius 4."""
    rng = np.random.default_rng(seed)
    sc = gaussian_cloud_scene(rng, n, sh_degree=3)
    cams = ring_cameras(n_views, 4.0, width=res, height=res, fx=fx)
    tgt = random_target(rng, n_views, res, res)
    return Workload(f"full-{n // 1000}k-sh3-{res}px-{n_views}v", sc, cams, 0, tgt)


def local_change(seed=3, n=1_000_000, n_views=16, width=1280, height=720, fx=1280.0,
                 radius=0.4, reinit="sfm", center=(0.0, 0.0, 0.0)) -> Workload:
    """1M Gaussians as in ``tiny``; the Gaussians within ``radius`` of ``center`` (the
    origin by default) form the change set and are re-initialised, then the scene is
    reordered static-first.  16 ring views of 1280x720.  ``scene_gt`` holds the
    unchanged scene in the same order (its renders are the targets)."""
    rng = np.random.default_rng(seed)
    gt = uniform_cube_scene(rng, n, sh_degree=0)
    c = np.asarray(center, dtype=np.float64).reshape(3, 1)
    active = np.linalg.norm(gt.means.astype(np.float64) - c, axis=0) <= radius
    gt_sorted, a0, perm = static_first(gt, active)
    idx = np.arange(a0, n)
    if reinit == "sfm":
        start = reinit_like_new_points(np.random.default_rng(33), gt_sorted, idx)
    else:   # same distribution as the rest of the scene
        r2 = np.random.default_rng(33)
        fresh = uniform_cube_scene(r2, len(idx), sh_degree=0, extent=radius)
        start = gt_sorted.copy()
        for a, b in zip(start.param_arrays(), fresh.param_arrays()):
            a[..., a0:] = b
    cams = ring_cameras(n_views, 4.0, width=width, height=height, fx=fx)
    tag = "" if not np.any(c) else "-c" + ",".join(f"{x:g}" for x in c.ravel())
    return Workload(f"local-{n // 1000}k-{width}x{height}-{n_views}v{tag}", start, cams, a0, None, gt_sorted,
                    {"perm": perm})


def fd_scene(seed=44, n=500, res=64, sh_degree=3) -> Workload:
    """500 Gaussians as in ``tiny`` with SH degree 3 coefficients N(0, 0.3), one 64x64
    view, fx = fy = 64, camera at distance 4."""
    rng = np.random.default_rng(seed)
    sc = uniform_cube_scene(rng, n, sh_degree=sh_degree)
    cam = Camera(np.eye(3), (0.0, 0.0, 4.0), res, res, res / 2.0, res / 2.0, res, res)
    tgt = random_target(rng, 1, res, res)
    return Workload(f"fd-{n}-sh{sh_degree}-{res}px", sc, [cam], 0, tgt)


def differentiation(seed=4, n=3_000_000, width=1920, height=1080, fx=1485.0) -> Workload:
    """3M Gaussians (N(0, 1.5^2 I) cloud, SH degree 3), batch of 4 ring views
    (0, 90, 180, 270 degrees) of 1920x1080."""
    rng = np.random.default_rng(seed)
    sc = gaussian_cloud_scene(rng, n, sh_degree=3)
    cams = ring_cameras(4, 4.0, width=width, height=height, fx=fx)
    tgt = random_target(rng, 4, height, width)
    return Workload(f"diff-{n // 1000}k-sh3-{width}x{height}-4v", sc, cams, 0, tgt)


RESOLUTIONS = ((640, 480), (1280, 720), (1920, 1080))


def serving_history(seed=5, n_base=2_000_000, n_steps=7, delta_range=(20_000, 100_000)):
    """A base scene plus ``n_steps`` change steps.  Step k picks a sphere around a random
    centre holding n_k ~ U{delta_range} Gaussians of the previous state, re-initialises
    them as new points, and records the step the way the paper's history store does
    (Supp. "History Recovery"): the 0/1 indicator I^k over the previous state and the
    previous values of the changed Gaussians O^k, stored before the change is applied.
    Returns (states, history) where ``states[k]`` is the full scene at timestep k
    (k = 0 is the base; each later state is static-first) and ``history[k-1]`` the
    (indicator, old changed Gaussians) pair of step k."""
    rng = np.random.default_rng(seed)
    base = gaussian_cloud_scene(rng, n_base, sh_degree=3)
    states = [base]
    history = []
    cur = base
    for _ in range(n_steps):
        nk = int(rng.integers(delta_range[0], delta_range[1] + 1))
        c = rng.normal(size=(3, 1))
        d = np.linalg.norm(cur.means.astype(np.float64) - c, axis=0)
        sel = np.argpartition(d, nk)[:nk]
        ind = np.zeros(cur.n, dtype=bool)
        ind[sel] = True
        reordered, a0, perm = static_first(cur, ind)
        nxt = reinit_like_new_points(rng, reordered, np.arange(a0, cur.n))
        history.append((ind, reordered.take(np.arange(a0, cur.n))))
        states.append(nxt)
        cur = nxt
    return states, history

"""CPU reference ("oracle") for the differentiable Gaussian-splatting hot path.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package; the GPU library never does.  It shares no
code with the GPU path: the renderer is plain C in ``oracle.c`` (double precision, brute
force over all Gaussians per pixel, no tiles), the loss gradient and Adam are written
below in numpy float64, and the binning reference is plain numpy on the GPU's own
float32 screen-space outputs.

Pins (see ``tests/test_oracle_*.py``): closed-form images of one and two Gaussians, the
stop-rule stack, spherical-harmonic orthonormality by quadrature, the EWA Jacobian and
covariance against central differences, compositing invariants, and finite-difference
gradients on tiny scenes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "liboracle.so"

# ------------------------------------------------------------------ build / load
_lib = None


def build(force: bool = True) -> Path:
    """Compile ``oracle.c`` with gcc (OpenMP, no floating-point contraction)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-Wall",
               "-o", str(tmp), str(_SRC), "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build()
        L = ctypes.CDLL(str(_LIB))
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int32)
        i64 = ctypes.c_int64
        L.orc_sh_basis.argtypes = [dp, dp]
        L.orc_sh_basis.restype = None
        L.orc_preprocess.argtypes = [i64, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, fp, ip]
        L.orc_preprocess.restype = ctypes.c_int
        L.orc_render.argtypes = [i64, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, i64, ip, dp, dp, ip, ip,
                                 dp, dp, dp, ip, dp, dp]
        L.orc_render.restype = ctypes.c_int
        L.orc_preprocess_backward.argtypes = [i64, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp,
                                              ctypes.c_int]
        L.orc_preprocess_backward.restype = ctypes.c_int
        L.orc_error_bounds.argtypes = [i64, ctypes.c_int, dp, dp, dp, dp, dp, dp, dp]
        L.orc_error_bounds.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, ct=ctypes.c_double):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------------ inputs
def cam_vec(cam) -> np.ndarray:
    """18 doubles: R (row-major), t, fx, fy, cx, cy, width, height."""
    v = np.zeros(18, dtype=np.float64)
    v[:9] = np.asarray(cam.R, dtype=np.float64).reshape(9)
    v[9:12] = np.asarray(cam.t, dtype=np.float64)
    v[12:16] = [cam.fx, cam.fy, cam.cx, cam.cy]
    v[16:18] = [cam.width, cam.height]
    return v


def _scene_args(scene, params=None):
    """Raw parameters as float64 arrays.  ``params`` may override them (a tuple of
    means, log_scales, quats, opacity_logit, sh already in float64), which the
    finite-difference tests use."""
    if params is None:
        params = tuple(_f64(a) for a in scene.param_arrays())
    return params


# ------------------------------------------------------------------ renderer
PP_FIELDS = ("u", "v", "A", "B", "C", "opacity", "r", "g", "b", "rx", "ry", "cov_a", "cov_b", "cov_c", "depth")
F_VISIBLE, F_CLAMPX, F_CLAMPY, F_SHCLAMP_R, F_SHCLAMP_G, F_SHCLAMP_B, F_NEAR = 1, 2, 4, 8, 16, 32, 64


def sh_basis(dirs) -> np.ndarray:
    """Real SH basis (degree <= 3, 16 values) at unit directions ``dirs`` [M, 3]."""
    dirs = _f64(np.atleast_2d(dirs))
    out = np.zeros((dirs.shape[0], 16))
    L = lib()
    for i in range(dirs.shape[0]):
        row = np.ascontiguousarray(dirs[i])
        o = np.zeros(16)
        L.orc_sh_basis(_p(row), _p(o))
        out[i] = o
    return out


def preprocess(scene, cam, params=None) -> dict:
    """Per-Gaussian screen-space quantities for one camera (double precision), the
    float32 depth key and decision flags."""
    n = scene.n
    args = _scene_args(scene, params)
    out = np.zeros((n, 16))
    z32 = np.zeros(n, dtype=np.float32)
    flags = np.zeros(n, dtype=np.int32)
    rc = lib().orc_preprocess(n, scene.sh_degree, *[_p(a) for a in args], _p(cam_vec(cam)), _p(out),
                              _p(z32, ctypes.c_float), _p(flags, ctypes.c_int32))
    assert rc == 0, rc
    res = {k: out[:, i] for i, k in enumerate(PP_FIELDS)}
    res["z32"] = z32
    res["flags"] = flags
    res["visible"] = (flags & F_VISIBLE) != 0
    return res


def error_bounds(scene, cam, params=None) -> dict:
    """Per-Gaussian bounds on the error of a float32 evaluation of the projected
    quantities (see err_bounds in oracle.c): ``u``, ``v`` (pixels), ``K`` (each conic
    entry), ``rgb`` [N, 3], ``cov`` (each screen-covariance entry) and ``det`` (relative
    error of the conic from the rounding of its inversion); zero for culled Gaussians."""
    n = scene.n
    args = _scene_args(scene, params)
    out = np.zeros((n, 8))
    rc = lib().orc_error_bounds(n, scene.sh_degree, *[_p(a) for a in args], _p(cam_vec(cam)), _p(out))
    assert rc == 0, rc
    return {"u": out[:, 0], "v": out[:, 1], "K": out[:, 2], "rgb": out[:, 3:6], "cov": out[:, 6], "det": out[:, 7]}


def all_pixels(width, height) -> np.ndarray:
    ys, xs = np.mgrid[0:height, 0:width]
    return np.stack([xs.ravel(), ys.ravel()], axis=1).astype(np.int32)


def render(scene, cam, bg=(0.0, 0.0, 0.0), pixels=None, dL_dC=None, params=None, pert=None) -> dict:
    """Brute-force render of ``pixels`` ([M, 2] int (px, py); default: the whole image).

    Returns ``rgb`` [M, 3], ``T`` [M], ``ncontrib`` [M], ``flag`` [M] and, for a full
    image, ``image`` [3, H, W].  With ``dL_dC`` ([M, 3], or [3, H, W] for a full image)
    it also returns the screen-space gradient ``grad2d`` [N, 9] (u, v, A, B, C, opacity,
    r, g, b), the absolute-term sums ``s2d`` [N, 9], the bound ``e2d`` [N, 9] on the
    float32 rounding of the compositing chains (see orc_render) and ``gflag`` [N].
    ``pert`` ([N, 9] in [-1, 1]) shifts each Gaussian's projected quantities by that
    fraction of their float32 error bounds before rendering."""
    n = scene.n
    full = pixels is None
    if full:
        pixels = all_pixels(cam.width, cam.height)
    pixels = np.ascontiguousarray(pixels, dtype=np.int32)
    m = pixels.shape[0]
    args = _scene_args(scene, params)
    rgb = np.zeros((m, 3))
    T = np.zeros(m)
    nc = np.zeros(m, dtype=np.int32)
    flag = np.zeros(m, dtype=np.int32)
    grad2d = s2d = gflag = e2d = None
    dl = None
    if dL_dC is not None:
        dl = _f64(dL_dC)
        if full and dl.ndim == 3:
            dl = np.ascontiguousarray(dl.reshape(3, -1).T)
        assert dl.shape == (m, 3)
        grad2d = np.zeros((n, 9))
        s2d = np.zeros((n, 9))
        e2d = np.zeros((n, 9))
    gflag = np.zeros(n, dtype=np.int32)
    bgv = _f64(bg)
    rc = lib().orc_render(n, scene.sh_degree, *[_p(a) for a in args], _p(cam_vec(cam)), _p(bgv), m,
                          _p(pixels, ctypes.c_int32), _p(rgb), _p(T), _p(nc, ctypes.c_int32),
                          _p(flag, ctypes.c_int32), _p(dl), _p(grad2d), _p(s2d), _p(gflag, ctypes.c_int32),
                          _p(e2d), _p(None if pert is None else _f64(pert)))
    assert rc == 0, rc
    res = {"rgb": rgb, "T": T, "ncontrib": nc, "flag": flag, "gflag": gflag}
    if full:
        res["image"] = rgb.T.reshape(3, cam.height, cam.width)
        res["T_image"] = T.reshape(cam.height, cam.width)
    if grad2d is not None:
        res["grad2d"] = grad2d
        res["s2d"] = s2d
        res["e2d"] = e2d
    return res


def n_raw(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


def split_raw(g: np.ndarray, sh_degree: int) -> dict:
    """[N, P] raw-parameter rows -> arrays in the scene's SoA layout."""
    K = (sh_degree + 1) ** 2
    n = g.shape[0]
    return {
        "means": np.ascontiguousarray(g[:, 0:3].T),
        "log_scales": np.ascontiguousarray(g[:, 3:6].T),
        "quats": np.ascontiguousarray(g[:, 6:10].T),
        "opacity_logit": np.ascontiguousarray(g[:, 10]),
        "sh": np.ascontiguousarray(g[:, 11:].reshape(n, K, 3).transpose(1, 2, 0)),
    }


def preprocess_backward(scene, cam, grad2d, s2d=None, params=None, e2d=None) -> dict:
    """Raw-parameter gradients (SoA dict) from a screen-space gradient [N, 9]; with
    ``s2d`` also the absolute-term bound ``s`` of each entry (same layout, key
    ``"s"``: ``s2d`` carried through the chain rule evaluated on absolute values, the
    size of the terms a float32 evaluation rounds before they cancel); with ``e2d`` (a
    screen-space error bound) that bound carried to the raw parameters through the
    absolute values of the exact Jacobian (key ``"e"``)."""
    n = scene.n
    P = n_raw(scene.sh_degree)
    args = _scene_args(scene, params)
    g = np.zeros((n, P))
    sr = np.zeros((n, P)) if s2d is not None else None
    rc = lib().orc_preprocess_backward(n, scene.sh_degree, *[_p(a) for a in args], _p(cam_vec(cam)),
                                       _p(_f64(grad2d)), _p(None if s2d is None else _f64(s2d)), _p(g), _p(sr), 1)
    assert rc == 0, rc
    res = split_raw(g, scene.sh_degree)
    if sr is not None:
        res["s"] = split_raw(sr, scene.sh_degree)
    if e2d is not None:
        er = np.zeros((n, P))
        scratch = np.zeros((n, P))
        rc = lib().orc_preprocess_backward(n, scene.sh_degree, *[_p(a) for a in args], _p(cam_vec(cam)),
                                           _p(_f64(grad2d)), _p(_f64(e2d)), _p(scratch), _p(er), 0)
        assert rc == 0, rc
        res["e"] = split_raw(er, scene.sh_degree)
    return res


# The float32 error term of the gradient comparison (see ``gradients``): renders with
# PERTURB_PATTERNS random sign patterns, and PERTURB_FACTOR times the largest deviation.
PERTURB_PATTERNS = 4
PERTURB_FACTOR = 2.0


def gradients(scene, cams, dL_dC_views, bg=(0.0, 0.0, 0.0), pixels=None, params=None,
              perturb=PERTURB_PATTERNS, seed=0) -> dict:
    """Raw-parameter gradients summed over views (``dL_dC_views[v]`` as for
    ``render``).  Returns the SoA gradient dict with the ``s`` sums, ``gflag`` and the
    float32 error term ``e`` of each entry:

    * the rounding of the compositing chains (``e2d`` of ``render``) carried to the raw
      parameters through the absolute value of the chain rule, plus
    * PERTURB_FACTOR times the largest change of the gradient when every Gaussian's
      projected quantities are moved by plus or minus their float32 error bounds, with
      ``perturb`` random sign patterns (seeded by ``seed``): a first-order estimate of
      how far a float32 evaluation of the same definition lands, with each pixel's
      contribution entering with its sign, as in the sum itself.

    ``perturb=0`` skips the perturbed renders (``e`` then holds the chain term only)."""
    total = None
    stot = etot = None
    gflag = np.zeros(scene.n, dtype=np.int32)
    for v, cam in enumerate(cams):
        pix = None if pixels is None else pixels[v]
        r = render(scene, cam, bg, pix, dL_dC_views[v], params)
        g = preprocess_backward(scene, cam, r["grad2d"], r["s2d"], params, e2d=r["e2d"])
        s = g.pop("s")
        e = g.pop("e")
        if total is None:
            total, stot, etot = g, s, e
        else:
            for k in total:
                total[k] = total[k] + g[k]
                stot[k] = stot[k] + s[k]
                etot[k] = etot[k] + e[k]
        gflag |= r["gflag"]
    total["s"] = stot
    if perturb:
        rng = np.random.default_rng(seed)
        dev = None
        for _ in range(perturb):
            gp = None
            for v, cam in enumerate(cams):
                pix = None if pixels is None else pixels[v]
                pert = rng.choice(np.array([-1.0, 1.0]), size=(scene.n, 9))
                r = render(scene, cam, bg, pix, dL_dC_views[v], params, pert=pert)
                g = preprocess_backward(scene, cam, r["grad2d"], None, params)
                gp = g if gp is None else {k: gp[k] + g[k] for k in gp}
            d = {k: np.abs(gp[k] - total[k]) for k in gp}
            dev = d if dev is None else {k: np.maximum(dev[k], d[k]) for k in d}
        for k in etot:
            etot[k] = etot[k] + PERTURB_FACTOR * dev[k]
    total["e"] = etot
    total["gflag"] = gflag
    return total


# ------------------------------------------------------------------ loss
def l1_loss_grad(image, target, pixel_mask=None):
    """L1 photometric loss L = sum|C - C*| / (3HW) over the whole image and its gradient
    sign(C - C*)/(3HW) (sign(0) = 0).  With ``pixel_mask`` ([H, W] bool) the gradient is
    zero outside the mask but keeps the full-image normalisation, and the loss sums only
    masked pixels."""
    image = _f64(image)
    target = _f64(target)
    c, h, w = image.shape[-3:]
    norm = 1.0 / (3.0 * h * w)
    diff = image - target
    grad = np.sign(diff) * norm
    absd = np.abs(diff)
    if pixel_mask is not None:
        grad = grad * pixel_mask
        absd = absd * pixel_mask
    return absd.sum() * norm, grad


# ------------------------------------------------------------------ Adam
def adam_step(params, grads, m, v, step, lrs, beta1=0.9, beta2=0.999, eps=1e-15, rows=None):
    """Adam (Kingma & Ba) on the rows ``rows`` (index array or slice over the last
    axis) of every parameter group; other rows are returned unchanged.  ``params``,
    ``grads``, ``m``, ``v`` are dicts of arrays whose last axis is the Gaussian index;
    ``lrs`` maps group -> learning rate; ``step`` is the 1-based step count.  Returns
    new (params, m, v) in float64."""
    if rows is None:
        rows = slice(None)
    bc1 = 1.0 - beta1 ** step
    bc2 = 1.0 - beta2 ** step
    P, M, V = {}, {}, {}
    for k in params:
        p = _f64(params[k]).copy()
        mm = _f64(m[k]).copy()
        vv = _f64(v[k]).copy()
        g = _f64(grads[k])[..., rows]
        mm[..., rows] = beta1 * mm[..., rows] + (1.0 - beta1) * g
        vv[..., rows] = beta2 * vv[..., rows] + (1.0 - beta2) * g * g
        mhat = mm[..., rows] / bc1
        vhat = vv[..., rows] / bc2
        p[..., rows] = p[..., rows] - lrs[k] * mhat / (np.sqrt(vhat) + eps)
        P[k], M[k], V[k] = p, mm, vv
    return P, M, V


# ------------------------------------------------------------------ binning reference
TILE = 16


def tile_grid(width, height):
    return (width + TILE - 1) // TILE, (height + TILE - 1) // TILE


def tile_rects(u, v, rx, ry, width, height):
    """Tile rectangle [x0, x1) x [y0, y1) of each Gaussian from its float32 screen
    centre and half extents: every pixel whose centre lies in [u - rx, u + rx] x
    [v - ry, v + ry] is covered.  Evaluated in float32 in this exact order:
    x0 = clamp(floor((u - rx - 0.5) * 0.0625), 0, TX), x1 = clamp(floor((u + rx - 0.5) *
    0.0625) + 1, 0, TX), and the same for y."""
    f = np.float32
    TX, TY = tile_grid(width, height)
    u, v, rx, ry = (np.asarray(a, dtype=np.float32) for a in (u, v, rx, ry))
    with np.errstate(invalid="ignore", over="ignore"):
        x0 = np.floor(((u - rx) - f(0.5)) * f(0.0625))
        x1 = np.floor(((u + rx) - f(0.5)) * f(0.0625)) + f(1.0)
        y0 = np.floor(((v - ry) - f(0.5)) * f(0.0625))
        y1 = np.floor(((v + ry) - f(0.5)) * f(0.0625)) + f(1.0)
    cl = lambda a, hi: np.minimum(np.maximum(a, f(0.0)), f(hi)).astype(np.int64)
    return cl(x0, TX), cl(x1, TX), cl(y0, TY), cl(y1, TY)


def bin_reference(u, v, rx, ry, z32, visible, width, height, active=None, use_mask=False):
    """Per-tile depth-ordered Gaussian lists for one view, from float32 inputs.

    Every visible Gaussian is emitted into each tile of its rectangle (only tiles of the
    render mask when ``use_mask``; the mask is the union of the rectangles of the
    visible Gaussians in ``active`` = (begin, end)), in Gaussian-index order; pairs are
    stably ordered by (tile, depth key bits), so equal depths stay in index order.
    Returns dict(values, tiles, ranges [T, 2], mask [T] bool, n_pairs, rects)."""
    TX, TY = tile_grid(width, height)
    T = TX * TY
    n = len(u)
    x0, x1, y0, y1 = tile_rects(u, v, rx, ry, width, height)
    vis = np.asarray(visible, dtype=bool)
    mask = np.ones(T, dtype=bool)
    if use_mask:
        mask = np.zeros(T, dtype=bool)
        a0, a1 = (0, n) if active is None else active
        for i in range(a0, a1):
            if vis[i] and x1[i] > x0[i] and y1[i] > y0[i]:
                yy, xx = np.mgrid[y0[i]:y1[i], x0[i]:x1[i]]
                mask[(yy * TX + xx).ravel()] = True
    gids, tiles = [], []
    for i in range(n):
        if not vis[i] or x1[i] <= x0[i] or y1[i] <= y0[i]:
            continue
        yy, xx = np.mgrid[y0[i]:y1[i], x0[i]:x1[i]]
        t = (yy * TX + xx).ravel()
        t = t[mask[t]]
        gids.append(np.full(t.shape, i, dtype=np.int64))
        tiles.append(t)
    gids = np.concatenate(gids) if gids else np.zeros(0, dtype=np.int64)
    tiles = np.concatenate(tiles) if tiles else np.zeros(0, dtype=np.int64)
    zbits = np.asarray(z32, dtype=np.float32).view(np.uint32).astype(np.int64)[gids]
    order = np.lexsort((gids, zbits, tiles))
    gids, tiles = gids[order], tiles[order]
    ranges = np.zeros((T, 2), dtype=np.int64)
    if len(tiles):
        starts = np.searchsorted(tiles, np.arange(T), side="left")
        ends = np.searchsorted(tiles, np.arange(T), side="right")
        nonempty = ends > starts
        ranges[nonempty, 0] = starts[nonempty]
        ranges[nonempty, 1] = ends[nonempty]
    return {"values": gids, "tiles": tiles, "ranges": ranges, "mask": mask, "n_pairs": len(gids),
            "rects": (x0, x1, y0, y1)}


def tile_list_reference(u, v, rx, ry, z32, visible, width, height, tile):
    """The depth-ordered Gaussian list of one tile (for spot checks at full size)."""
    TX, _ = tile_grid(width, height)
    x0, x1, y0, y1 = tile_rects(u, v, rx, ry, width, height)
    tx, ty = tile % TX, tile // TX
    sel = np.nonzero(np.asarray(visible, bool) & (x0 <= tx) & (tx < x1) & (y0 <= ty) & (ty < y1))[0]
    zbits = np.asarray(z32, dtype=np.float32).view(np.uint32)[sel].astype(np.int64)
    return sel[np.lexsort((sel, zbits))]


# ------------------------------------------------------------------ change region: spheres
# Supp. "Identifying Changed 3D Regions via Majority Voting": one sphere per cluster of
# changed Gaussians, centred on the cluster's mean, radius 1.1 times the 98th percentile
# of the distances to it; Supp. "3DGS Optimization in Changed Regions": every 15
# iterations, changed Gaussians whose centre lies outside every sphere are removed.
SPHERE_QUANTILE = 0.98
SPHERE_SCALE = 1.1


def fit_spheres(means, labels, n_spheres):
    """Centres [S, 3] and radii [S] (float64) of the clusters of ``means`` ([3, M]) given
    by ``labels`` ([M] int; -1: in no cluster).  The percentile interpolates linearly
    between the order statistics at positions floor(q) and floor(q) + 1 of the sorted
    distances, q = 0.98 (c - 1) for a cluster of c points.  An empty cluster gets centre
    0 and radius -1 (it contains nothing)."""
    means = _f64(means)
    labels = np.asarray(labels)
    centers = np.zeros((n_spheres, 3))
    radii = np.full(n_spheres, -1.0)
    for s in range(n_spheres):
        pts = means[:, labels == s]
        c = pts.shape[1]
        if c == 0:
            continue
        m = pts.sum(axis=1) / c
        d = np.sort(np.sqrt(((pts - m[:, None]) ** 2).sum(axis=0)))
        q = SPHERE_QUANTILE * (c - 1)
        lo = int(np.floor(q))
        hi = min(lo + 1, c - 1)
        centers[s] = m
        radii[s] = SPHERE_SCALE * (d[lo] + (q - lo) * (d[hi] - d[lo]))
    return centers, radii


def sphere_keep(means, centers, radii):
    """Whether each centre ([3, M]) lies in the union of the spheres: |mu - m| <= r for
    some sphere (the boundary counts as inside).  The decision is taken in float32, in
    this order, with every operation rounded: d = mu - m per axis, d2 = (dx dx + dy dy) +
    dz dz, inside iff d2 <= r r, so that a float32 implementation takes the same
    decisions; spheres with a negative radius contain nothing."""
    f = np.float32
    mu = np.asarray(means, dtype=f)
    keep = np.zeros(mu.shape[1], dtype=bool)
    for m, r in zip(np.asarray(centers, dtype=f), np.asarray(radii, dtype=f)):
        if r < 0:
            continue
        dx, dy, dz = mu[0] - m[0], mu[1] - m[1], mu[2] - m[2]
        d2 = (dx * dx + dy * dy) + dz * dz
        keep |= d2 <= r * r
    return keep


def compact_rows(arrays, keep, begin):
    """The parameter arrays (last axis = Gaussian) with the rows [begin, N) whose
    ``keep`` ([N - begin] bool) is false removed: rows before ``begin`` stay where they
    are and the kept rows follow in their order, so the changed Gaussians stay the
    contiguous suffix (Supp. "History Recovery")."""
    keep = np.asarray(keep, dtype=bool)
    out = []
    for a in arrays:
        a = np.asarray(a)
        out.append(np.concatenate([a[..., :begin], a[..., begin:][..., keep]], axis=-1))
    return out


# ------------------------------------------------------------------ change lifting
# Supp. "Detecting Changes in 2D": the binary change masks are dilated by 2% of the image
# width, by a convolution with a kernel of ones and a threshold at 0.  Supp.
# "Identifying Changed 3D Regions via Majority Voting": each Gaussian's centre is
# projected into every view; c_i counts the views whose mask holds it, o_i those whose
# image it falls outside; g_i is changed iff 4/3 o_i < |I| < 2 c_i.
DILATE_FRACTION = 0.02


def dilation_radius(width):
    """Half-width of the square dilation kernel: 2% of the image width, rounded to the
    nearest pixel (halves up)."""
    return int(np.floor(DILATE_FRACTION * width + 0.5))


def dilate_masks(masks, radius):
    """masks [V, H, W] (0/1) -> [V, H, W] uint8: 1 where the sum of the mask over the
    (2 radius + 1)^2 square around the pixel (pixels outside the image count 0) is > 0.
    The sums are exact integer box sums of the mask's integral image."""
    m = (np.asarray(masks) != 0).astype(np.int64)
    V, H, W = m.shape
    S = np.zeros((V, H + 1, W + 1), dtype=np.int64)
    S[:, 1:, 1:] = m.cumsum(1).cumsum(2)
    y0 = np.clip(np.arange(H) - radius, 0, H)
    y1 = np.clip(np.arange(H) + radius + 1, 0, H)
    x0 = np.clip(np.arange(W) - radius, 0, W)
    x1 = np.clip(np.arange(W) + radius + 1, 0, W)
    box = (S[:, y1][:, :, x1] - S[:, y0][:, :, x1] - S[:, y1][:, :, x0] + S[:, y0][:, :, x0])
    return np.ascontiguousarray(box > 0).astype(np.uint8)


def project_centres_f32(means, cam):
    """Pixel coordinates (u, v) and depth Z of the centres ([3, N]) in float32, every
    operation rounded, in this order: X = ((R00 x + R01 y) + R02 z) + t0 (Y, Z alike),
    u = (fx X) / Z + cx, v = (fy Y) / Z + cy."""
    f = np.float32
    x, y, z = (np.asarray(means[k], dtype=f) for k in range(3))
    R = np.asarray(cam.R, dtype=f).reshape(3, 3)
    t = np.asarray(cam.t, dtype=f)
    P = [((R[a, 0] * x + R[a, 1] * y) + R[a, 2] * z) + t[a] for a in range(3)]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        u = (f(cam.fx) * P[0]) / P[2] + f(cam.cx)
        v = (f(cam.fy) * P[1]) / P[2] + f(cam.cy)
    return u, v, P[2]


def majority_vote(means, cams, masks):
    """(changed [N] bool, c [N], o [N]) for centres ``means`` [3, N], cameras ``cams``
    and masks [V, H, W]: a centre is outside view v when its depth is at most the near
    plane 0.2 or its pixel coordinates leave [0, W) x [0, H); otherwise it falls in
    pixel (floor(u), floor(v)) and counts for c when the mask is 1 there.  The
    projection is taken in float32 as ``project_centres_f32`` states (the precision of
    the GPU kernel, so both take the same decisions)."""
    masks = np.asarray(masks)
    n = np.asarray(means).shape[1]
    c = np.zeros(n, dtype=np.int64)
    o = np.zeros(n, dtype=np.int64)
    for v_, cam in enumerate(cams):
        u, v, Z = project_centres_f32(means, cam)
        inside = (Z > np.float32(0.2)) & (u >= 0) & (u < np.float32(cam.width)) & (v >= 0) & \
                 (v < np.float32(cam.height))
        o += ~inside
        px = np.where(inside, np.floor(np.where(inside, u, 0)), 0).astype(np.int64)
        py = np.where(inside, np.floor(np.where(inside, v, 0)), 0).astype(np.int64)
        c += inside & (masks[v_, py, px] != 0)
    V = len(cams)
    changed = (4 * o < 3 * V) & (V < 2 * c)
    return changed, c, o


# ------------------------------------------------------------------ history and merges
# Supp. "History Recovery": before optimising step t the Gaussians are reordered so the
# unchanged ones (I^t = 0) come first, and O^t (the changed Gaussians' values) and I^t
# are stored; G^{t-1} is rebuilt from G^t by putting the first #static Gaussians of G^t
# where I^t = 0 and O^t where I^t = 1 (alg:example).  Supp. "Batched Updates": two
# concurrent updates merge as the unchanged Gaussians of G^{t-1} followed by O_1 and O_2.
def reorder_static_first(arrays, indicator):
    """The rows (last axis) with indicator 0 in their order, then those with 1 in their
    order; returns (arrays, #static)."""
    ind = np.asarray(indicator, dtype=bool)
    order = np.concatenate([np.nonzero(~ind)[0], np.nonzero(ind)[0]])
    return [np.asarray(a)[..., order] for a in arrays], int((~ind).sum())


def recover_previous(latest, indicator, changed_before):
    """G^{k-1} from G^k (``latest``), I^k (``indicator``, over G^{k-1}) and O^k
    (``changed_before``): an array of the target size, O^k at the positions where I^k is
    1 and the first #static Gaussians of G^k, in order, where it is 0."""
    ind = np.asarray(indicator, dtype=bool)
    n_static = int((~ind).sum())
    out = []
    for g, o in zip(latest, changed_before):
        g, o = np.asarray(g), np.asarray(o)
        n = np.empty(g.shape[:-1] + (len(ind),), dtype=g.dtype)
        n[..., ind] = o
        n[..., ~ind] = g[..., :n_static]
        out.append(n)
    return out


def merge_updates(prev, ind1, ind2, o1, o2):
    """G^t = G^{t-1}[not I_1 and not I_2] followed by O_1 and O_2 (the unchanged
    Gaussians in their order, then both updates)."""
    keep = ~(np.asarray(ind1, dtype=bool) | np.asarray(ind2, dtype=bool))
    return [np.concatenate([np.asarray(p)[..., keep], np.asarray(a), np.asarray(b)], axis=-1)
            for p, a, b in zip(prev, o1, o2)]


# ------------------------------------------------------------------ L1 + D-SSIM loss
# The paper trains with the default 3D Gaussian Splatting loss (Supp. "Implementation
# Details"): (1 - lambda) L1 + lambda (1 - SSIM), lambda = 0.2, SSIM with an 11 x 11
# Gaussian window of standard deviation 1.5, C1 = 0.01^2, C2 = 0.03^2, computed per
# channel with zero padding at the image border and averaged over channels and pixels.
SSIM_SIZE = 11
SSIM_SIGMA = 1.5
SSIM_C1 = 0.01 ** 2
SSIM_C2 = 0.03 ** 2
LAMBDA_DSSIM = 0.2


def ssim_window():
    """The 11 x 11 window: outer product of the normalised 1D Gaussian exp(-i^2 / (2
    sigma^2)), i = -5..5."""
    i = np.arange(SSIM_SIZE) - SSIM_SIZE // 2
    g = np.exp(-(i * i) / (2.0 * SSIM_SIGMA ** 2))
    g /= g.sum()
    return np.outer(g, g)


def _window_sum(a, w):
    """sum over the window centred at each pixel of w(offset) a(pixel + offset), zero
    outside the image; a [..., H, W]."""
    r = w.shape[0] // 2
    H, W = a.shape[-2:]
    pad = np.zeros(a.shape[:-2] + (H + 2 * r, W + 2 * r))
    pad[..., r:r + H, r:r + W] = a
    out = np.zeros(a.shape)
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            out += w[dy + r, dx + r] * pad[..., r + dy:r + dy + H, r + dx:r + dx + W]
    return out


def ssim_map(x, y):
    """Per-pixel SSIM [..., H, W] of images x, y [..., H, W] (float64)."""
    x, y = _f64(x), _f64(y)
    w = ssim_window()
    mx, my = _window_sum(x, w), _window_sum(y, w)
    exx, eyy, exy = _window_sum(x * x, w), _window_sum(y * y, w), _window_sum(x * y, w)
    A = 2 * mx * my + SSIM_C1
    B = 2 * (exy - mx * my) + SSIM_C2
    C = mx * mx + my * my + SSIM_C1
    D = (exx - mx * mx) + (eyy - my * my) + SSIM_C2
    return A * B / (C * D)


def l1_dssim_loss_grad(image, target, lam=LAMBDA_DSSIM):
    """Loss (1 - lam) mean|x - y| + lam (1 - mean SSIM) over [3, H, W] images and its
    gradient with respect to x.  SSIM at pixel p is a function of its window sums
    mu_x, E[xx], E[xy] (and y's), so by the chain rule
    d SSIM(p) / d x(q) = w(q - p) [d/dmu_x + 2 x(q) d/dE[xx] + y(q) d/dE[xy]] SSIM(p),
    and the gradient at q is the window sum of those three partial maps, the zero padding
    making them vanish outside the image."""
    x, y = _f64(image), _f64(target)
    n = x.size
    w = ssim_window()
    mx, my = _window_sum(x, w), _window_sum(y, w)
    exx, eyy, exy = _window_sum(x * x, w), _window_sum(y * y, w), _window_sum(x * y, w)
    A = 2 * mx * my + SSIM_C1
    B = 2 * (exy - mx * my) + SSIM_C2
    C = mx * mx + my * my + SSIM_C1
    D = (exx - mx * mx) + (eyy - my * my) + SSIM_C2
    s = A * B / (C * D)
    # partials of s = A B / (C D) in (mu_x, E[xx], E[xy]) with A, B, C, D as above
    d_mx = (2 * my * B - 2 * my * A) / (C * D) - s * (2 * mx / C - 2 * mx / D)
    d_exx = -s / D
    d_exy = 2 * A / (C * D)
    g_ssim = _window_sum(d_mx, w) + 2 * x * _window_sum(d_exx, w) + y * _window_sum(d_exy, w)
    loss = (1 - lam) * np.abs(x - y).sum() / n + lam * (1 - s.sum() / n)
    grad = (1 - lam) * np.sign(x - y) / n - lam * g_ssim / n
    return loss, grad

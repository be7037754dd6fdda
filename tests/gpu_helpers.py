"""Shared helpers of the GPU parity tests: run the HIP path through the C-ABI and
compare with the CPU reference on the same seeded inputs."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_2506_21117_amd import api

# Tolerances (the oracle is float64, the GPU float32):
PIX_REL, PIX_ABS = 1e-4, 1e-6          # pixels
# gradients: rel + GRAD_S * (sum of |per-pixel terms|, the summation order of float
# atomics) + the oracle's float32 error term e (rounding of the projected quantities
# carried through the compositing, and of the compositing chains) + GRAD_ABS
GRAD_REL, GRAD_S = 1e-3, 1e-5
GRAD_ABS = 1e-10


def to_np(t):
    return t.detach().cpu().numpy()


def gpu_preprocess(g, cams, gather=None):
    proj = api.project_preprocess(g, cams, gather=gather)
    torch.cuda.synchronize()
    return proj


def unpack(proj, view):
    n = proj.n
    s = to_np(proj.splat)[view * n:(view + 1) * n]
    rect = to_np(proj.rect)[view * n:(view + 1) * n].view(np.uint32)
    return {
        "u": s[:, 0], "v": s[:, 1], "A": s[:, 2], "B": s[:, 3], "C": s[:, 4], "opacity": s[:, 5],
        "r": s[:, 6], "g": s[:, 7], "b": s[:, 8], "rx": s[:, 9], "ry": s[:, 10],
        "depth": to_np(proj.depth)[view * n:(view + 1) * n],
        "x0": rect[:, 0] & 0xFFFF, "x1": rect[:, 0] >> 16, "y0": rect[:, 1] & 0xFFFF, "y1": rect[:, 1] >> 16,
        "flags": to_np(proj.flags)[view * n:(view + 1) * n].view(np.uint32),
    }


def bin_reference_for(gp, cam, active=None, use_mask=False):
    return oracle.bin_reference(gp["u"], gp["v"], gp["rx"], gp["ry"], gp["depth"], (gp["flags"] & 1) != 0,
                                cam.width, cam.height, active=active, use_mask=use_mask)


def masked_pixels(bins, cam, view=0):
    """Pixel coordinates [M, 2] of the tiles of the render mask of one view."""
    TX, TY = api.tile_grid(cam.width, cam.height)
    words = to_np(bins.tile_mask).view(np.uint32)[view]
    tiles = [t for t in range(TX * TY) if (words[t // 32] >> (t % 32)) & 1]
    out = []
    for t in tiles:
        x0, y0 = (t % TX) * 16, (t // TX) * 16
        ys, xs = np.mgrid[y0:min(y0 + 16, cam.height), x0:min(x0 + 16, cam.width)]
        out.append(np.stack([xs.ravel(), ys.ravel()], 1))
    return np.concatenate(out).astype(np.int32) if out else np.zeros((0, 2), np.int32), tiles


def check_pixels(got_rgb, ref, what="", max_excused=1e-3):
    """got_rgb [M, 3] vs the oracle render dict of the same pixels.  A pixel outside the
    tolerance is excused only when the oracle flags it (one of its decisions lies within
    that decision's float32 error of its threshold, so a float32 evaluation may take it
    either way); excused pixels must be rare: at most a fraction ``max_excused``, or 3."""
    flagged = ref["flag"] != 0
    err = np.abs(got_rgb - ref["rgb"])
    tol = PIX_REL * np.abs(ref["rgb"]) + PIX_ABS
    fail = (err > tol).any(1)
    bad = fail & ~flagged
    assert not bad.any(), (f"{what}: {bad.sum()} pixels outside tolerance; worst err "
                           f"{err[bad].max():.3e} at ref {ref['rgb'][bad][np.argmax(err[bad].max(1))]}")
    excused = fail & flagged
    assert excused.mean() < max_excused or excused.sum() <= 3, (
        f"{what}: {excused.sum()} excused pixels of {len(excused)} ({flagged.sum()} flagged)")
    keep = ~excused
    return float(err[keep].max()) if keep.any() else 0.0


def check_grads(gpu: api.GaussianTensors, ref: dict, rows, what=""):
    """GPU gradients vs oracle gradients on the rows ``rows`` (slice or index array).
    Rows the oracle flags (near-threshold decisions at their pixels) are excused only
    when they fail; their number must stay small."""
    worst = 0.0
    excused = set()
    gflag = ref["gflag"]
    for k in api.GaussianTensors.NAMES:
        g = to_np(getattr(gpu, k)).astype(np.float64)[..., rows]
        o = ref[k][..., rows]
        s = ref["s"][k][..., rows]
        e = ref["e"][k][..., rows]
        err = np.abs(g - o)
        tol = GRAD_REL * np.abs(o) + GRAD_S * s + e + GRAD_ABS
        bad = err > tol
        if bad.any():
            axes = tuple(range(bad.ndim - 1))
            bad_rows = np.nonzero(bad.any(axis=axes) if axes else bad)[0]
            fl = gflag[rows][bad_rows] if not isinstance(rows, slice) else gflag[rows][bad_rows]
            unexcused = bad_rows[fl == 0]
            assert len(unexcused) == 0, (
                f"{what} {k}: {len(unexcused)} rows outside tolerance, e.g. row {unexcused[0]}: "
                f"gpu {g[..., unexcused[0]]} ref {o[..., unexcused[0]]} s {s[..., unexcused[0]]} "
                f"e {e[..., unexcused[0]]}")
            excused.update(bad_rows.tolist())
        r = err / (tol + 1e-30)
        worst = max(worst, float(r.max()) if r.size else 0.0)
    nrows = (rows.stop - rows.start) if isinstance(rows, slice) else len(rows)
    assert len(excused) <= max(2, 1e-3 * nrows), f"{what}: {len(excused)} rows excused"
    return worst

"""Parity of every hot-path call (through the C-ABI) with the CPU reference.

Binning is compared bit for bit against the reference binning run on the GPU's own
float32 screen-space outputs; pixels within 1e-4 relative; gradients within 1e-3
relative (plus the float32 summation-order term 1e-5 * sum of |per-pixel terms|);
preprocess outputs within float32 rounding; Adam within 1e-6 of the step size.
"""
import re
from pathlib import Path

import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_helpers import (bin_reference_for, check_grads, check_pixels, gpu_preprocess, masked_pixels, to_np,
                         unpack)
from paper_2506_21117_amd import api
from paper_2506_21117_amd._ffi import BINS_COMPLETE as COMPLETE

pytestmark = pytest.mark.gpu


# ------------------------------------------------------------------ workloads
def _clamp_scene(seed=13):
    """Gaussians off to the sides (Jacobian clamp), some behind the near plane, strong
    SH bands (colour clamp), 100x37 ragged image."""
    rng = np.random.default_rng(seed)
    n = 400
    means = np.stack([rng.uniform(-5, 5, n), rng.uniform(-2, 2, n), rng.uniform(-4.5, 1.5, n)]).astype(np.float32)
    ls = rng.normal(-1.8, 0.5, (3, n)).astype(np.float32)
    sh = rng.normal(0, 0.9, (4, 3, n)).astype(np.float32)
    sc = scenes.Scene(means, ls, rng.normal(size=(4, n)), rng.normal(0, 1.5, n), sh, 1)
    cam = scenes.Camera(np.eye(3), (0, 0, 4), 60, 60, 50, 18.5, 100, 37)
    return sc, [cam]


def workload(name):
    if name == "tiny":
        w = scenes.tiny()
        return w.scene, w.cameras
    if name == "sh3":
        w = scenes.fd_scene(n=500, res=64)
        return w.scene, w.cameras
    if name == "clamp":
        return _clamp_scene()
    if name == "ring2":
        w = scenes.full_scene(n=3000, n_views=2, res=96, fx=132.0)
        return w.scene, w.cameras
    raise KeyError(name)


CASES = ["tiny", "sh3", "clamp", "ring2"]


def _sliced_case(name):
    if name == "local":
        w = scenes.local_change(n=60_000, n_views=2, width=320, height=180, fx=320.0)
        return w.scene, w.cameras[:1], (w.active_begin, w.scene.n)
    if name == "cloud":
        w = scenes.full_scene(n=40_000, n_views=2, res=160, fx=220.0)
        return w.scene, w.cameras, (36_000, 40_000)
    sc, cams = workload(name)
    return sc, cams, (int(sc.n * 0.8), sc.n)


# ------------------------------------------------------------------ a1 preprocess
@pytest.mark.parametrize("case", CASES)
def test_preprocess_parity(dev, case):
    sc, cams = workload(case)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    for v, cam in enumerate(cams):
        gp = unpack(proj, v)
        ref = oracle.preprocess(sc, cam)
        near = (ref["flags"] & oracle.F_NEAR) != 0
        vis_g = (gp["flags"] & 1) != 0
        assert np.all((vis_g == ref["visible"]) | near)
        np.testing.assert_array_equal(gp["depth"].view(np.uint32), ref["z32"].view(np.uint32))
        both = vis_g & ref["visible"] & ~near
        assert both.sum() > 0.3 * sc.n or case == "clamp"

        def close(k, rel, abs_=0.0, scale=None):
            o = ref[k][both]
            s = np.abs(o) if scale is None else scale
            err = np.abs(gp[k][both].astype(np.float64) - o)
            assert np.all(err <= rel * s + abs_), (k, float((err / (rel * s + abs_)).max()))

        close("u", 2e-6, 1e-4)
        close("v", 2e-6, 1e-4)
        cn = np.sqrt(ref["A"] ** 2 + 2 * ref["B"] ** 2 + ref["C"] ** 2)[both]
        for k in ("A", "B", "C"):
            close(k, 1e-4, scale=cn)      # det = ac - b^2 cancels for thin ellipses
        close("opacity", 1e-6)
        for k in ("r", "g", "b"):
            close(k, 1e-6, 2e-6)
        close("rx", 1e-4, 1e-4)
        close("ry", 1e-4, 1e-4)
        clamp_bits = oracle.F_CLAMPX | oracle.F_CLAMPY | oracle.F_SHCLAMP_R | oracle.F_SHCLAMP_G | oracle.F_SHCLAMP_B
        np.testing.assert_array_equal(gp["flags"][both] & clamp_bits, ref["flags"][both] & clamp_bits)
        # the tile rectangle is the documented float32 formula of the GPU's own outputs
        x0, x1, y0, y1 = oracle.tile_rects(gp["u"], gp["v"], gp["rx"], gp["ry"], cam.width, cam.height)
        for a, b in ((gp["x0"], x0), (gp["x1"], x1), (gp["y0"], y0), (gp["y1"], y1)):
            np.testing.assert_array_equal(a[vis_g].astype(np.int64), b[vis_g])


def _same_projection(a, b):
    for k in ("splat", "depth", "rect", "flags"):
        np.testing.assert_array_equal(to_np(getattr(a, k)).view(np.uint32), to_np(getattr(b, k)).view(np.uint32))


@pytest.mark.parametrize("case", ["sh3", "ring2"])
def test_projecting_changed_rows_equals_full_projection(dev, case):
    """Re-projecting rows [a0, a1) after their parameters changed gives the full
    projection of the new parameters, bit for bit, and leaves the other rows alone."""
    sc, cams = workload(case)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    a0, a1 = sc.n // 3, 2 * sc.n // 3
    rng = np.random.default_rng(11)
    for k in api.GaussianTensors.NAMES:
        x = getattr(g, k)
        x[..., a0:a1] += torch.as_tensor(rng.normal(size=x[..., a0:a1].shape).astype(np.float32) * 0.05, device=dev)
    api.project_preprocess_rows(g, cams, (a0, a1), proj)
    _same_projection(proj, gpu_preprocess(g, cams))
    api.project_preprocess_rows(g, cams, (a1, a1), proj)   # an empty range writes nothing
    _same_projection(proj, gpu_preprocess(g, cams))


def test_local_steps_keep_each_views_projection_of_frozen_rows(dev):
    """The optimiser's local steps re-project only the change set of the step's view;
    afterwards every view's kept projection, its change set re-projected, equals a full
    projection of the current parameters (the frozen rows never changed).  The change
    ball sits on the cube face z = +1, so it is visible and the steps move it."""
    from paper_2506_21117_amd.optim import SplatOptimizer

    w = scenes.local_change(n=40_000, n_views=3, width=320, height=180, fx=320.0, radius=0.4, center=(0.0, 0.0, 1.0))
    a = (w.active_begin, w.scene.n)
    g = api.GaussianTensors.from_scene(w.scene, dev)
    frozen = {k: getattr(g, k)[..., :a[0]].clone() for k in api.GaussianTensors.NAMES}
    targets = torch.rand(3, 3, 180, 320, generator=torch.Generator(device=dev).manual_seed(2), device=dev)
    opt = SplatOptimizer(g, w.cameras, targets, active=a, local=True)
    assert opt.proj_views is not None
    for i in range(7):
        opt.step(i % 3)
    torch.cuda.synchronize()
    assert not opt.overflowed()
    for k in api.GaussianTensors.NAMES:
        np.testing.assert_array_equal(to_np(getattr(g, k)[..., :a[0]]), to_np(frozen[k]))
        moved = getattr(g, k)[..., a[0]:] != getattr(api.GaussianTensors.from_scene(w.scene, dev), k)[..., a[0]:]
        assert bool(moved.any()), k
    for v, cam in enumerate(w.cameras):
        api.project_preprocess_rows(g, [cam], a, opt.proj_views[v])
        _same_projection(opt.proj_views[v], gpu_preprocess(g, [cam]))


# ------------------------------------------------------------------ a2, a3 binning
def _check_bins(bins, proj, cams, active, use_mask):
    c = bins.read_counters()
    assert not c["overflow"]
    n = proj.n
    TX, TY = api.tile_grid(cams[0].width, cams[0].height)
    T = TX * TY
    values = to_np(bins.values).view(np.uint32)
    keys = to_np(bins.keys).view(np.uint32)
    ranges = to_np(bins.ranges).view(np.uint32).astype(np.int64)
    mask_words = to_np(bins.tile_mask).view(np.uint32)
    off = 0
    total_tiles = []
    for v, cam in enumerate(cams):
        gp = unpack(proj, v)
        ref = bin_reference_for(gp, cam, active, use_mask)
        P = ref["n_pairs"]
        np.testing.assert_array_equal(values[off:off + P].astype(np.int64), ref["values"] + v * n)
        np.testing.assert_array_equal(keys[off:off + P].astype(np.int64), ref["tiles"] + v * T)
        rv = ranges[v * T:(v + 1) * T]
        exp = ref["ranges"].copy()
        ne = exp[:, 1] > exp[:, 0]
        exp[ne] += off
        np.testing.assert_array_equal(rv, exp)
        bits = np.array([(mask_words[v][t // 32] >> (t % 32)) & 1 for t in range(T)], bool)
        np.testing.assert_array_equal(bits, ref["mask"])
        total_tiles += [v * T + t for t in np.nonzero(ref["mask"])[0]]
        off += P
    assert c["pairs"] == off == c["written"]
    np.testing.assert_array_equal(to_np(bins.tile_list)[:c["tiles"]], np.array(total_tiles, np.int64))
    return off


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("use_mask", [False, True])
def test_bin_and_sort_bit_exact(dev, case, use_mask):
    sc, cams = workload(case)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    active = (int(sc.n * 0.8), sc.n)
    bins = api.bin_and_sort(proj, cams, active, use_mask, capacity=200_000, mode=COMPLETE)
    torch.cuda.synchronize()
    P = _check_bins(bins, proj, cams, active, use_mask)
    assert P > 0


def test_bin_and_sort_many_tile_bits(dev):
    """3600 tiles per view (12 tile bits, two sort passes) plus views stacked (13 bits)."""
    w = scenes.full_scene(n=4000, n_views=2, res=960, fx=1320.0)
    cams = [scenes.Camera(c.R, c.t, 1280, 1280, 640, 360, 1280, 720) for c in w.cameras]
    g = api.GaussianTensors.from_scene(w.scene, dev)
    proj = gpu_preprocess(g, cams)
    for use_mask in (False, True):
        bins = api.bin_and_sort(proj, cams, (3000, 4000), use_mask, capacity=2_000_000, mode=COMPLETE)
        torch.cuda.synchronize()
        _check_bins(bins, proj, cams, (3000, 4000), use_mask)


@pytest.mark.parametrize("mode", [COMPLETE, api._ffi.BINS_DEPTH_SLICED, api._ffi.BINS_DEPTH_SLICED_LOCAL])
def test_counting_placement_with_more_than_1024_masked_tiles(dev, mode):
    """One 1280x720 view whose render mask covers more than 1 024 of its 3 600 tiles: the
    counting placement's layout for that many tile slots (masks and scans without the
    LDS copies of the corner table), against the reference bit for bit, and complete
    and depth-sliced lists giving the same image."""
    w = scenes.full_scene(n=4000, n_views=1, res=960, fx=1320.0)
    cams = [scenes.Camera(c.R, c.t, 1280, 1280, 640, 360, 1280, 720) for c in w.cameras]
    g = api.GaussianTensors.from_scene(w.scene, dev)
    proj = gpu_preprocess(g, cams)
    active = (1000, 4000)
    bins = api.bin_and_sort(proj, cams, active, True, capacity=2_000_000, mode=mode)
    img, T, nc = api.render_forward(proj, bins, cams)
    torch.cuda.synchronize()
    c = bins.read_counters()
    assert c["tiles"] > 1024, c["tiles"]
    if mode == COMPLETE:
        _check_bins(bins, proj, cams, active, True)
    else:
        ref = api.bin_and_sort(proj, cams, active, True, capacity=2_000_000, mode=COMPLETE)
        img_c, T_c, nc_c = api.render_forward(proj, ref, cams)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(to_np(img), to_np(img_c))
        np.testing.assert_array_equal(to_np(nc), to_np(nc_c))


def test_counting_placement_without_kept_masks(dev):
    """A slab whose chunks x tile slots exceed the kept-mask budget (over 150 000 entries
    of one view, all in the first slab of complete lists, over more than 3 000 tiles:
    2 344 x 3 600 > 8 Mi words) makes the emission build its tile masks again: its image
    and contributor counts equal those of depth-sliced lists, whose first slab keeps its
    masks."""
    w = scenes.full_scene(n=350_000, n_views=1, res=960, fx=1320.0)
    cams = [scenes.Camera(c.R, c.t, 1280, 1280, 640, 360, 1280, 720) for c in w.cameras]
    g = api.GaussianTensors.from_scene(w.scene, dev)
    proj = gpu_preprocess(g, cams)
    out = []
    for mode in (COMPLETE, api._ffi.BINS_DEPTH_SLICED):
        bins = api.bin_and_sort(proj, cams, (0, 350_000), True, capacity=60_000_000, mode=mode)
        img, T, nc = api.render_forward(proj, bins, cams)
        torch.cuda.synchronize()
        c = bins.read_counters()
        assert not c["overflow"] and c["tiles"] > 3000
        out.append((to_np(img), to_np(nc), c))
    c0 = out[0][2]
    assert ((c0["entries"] + 63) // 64) * c0["tiles"] > 8 << 20, c0
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_capacity_overflow_is_reported_and_recoverable(dev):
    sc, cams = workload("tiny")
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    small = api.bin_and_sort(proj, cams, capacity=100, mode=COMPLETE)
    c = small.read_counters()
    assert c["overflow"] and c["pairs"] > 100 and c["written"] == 0 and c["tiles"] == 0
    assert to_np(small.counters)[5] == 1            # sticky
    img, _, _ = api.render_forward(proj, small, cams)   # renders nothing, touches nothing
    torch.cuda.synchronize()
    assert float(img.abs().sum()) == 0.0
    big = api.bin_and_sort(proj, cams, capacity=c["pairs"], mode=COMPLETE)
    torch.cuda.synchronize()
    _check_bins(big, proj, cams, None, False)
    # depth-sliced lists: an overflow in the first slab ...
    sl = api.bin_and_sort(proj, cams, capacity=c["pairs"] // 3)
    api.render_forward(proj, sl, cams)
    assert sl.read_counters()["overflow"] and to_np(sl.counters)[5] == 1
    # ... and in the second (a sparse cloud: more than one slab, edge tiles still alive)
    sc2, cams2, _ = _sliced_case("cloud")
    proj2 = gpu_preprocess(api.GaussianTensors.from_scene(sc2, dev), cams2)
    ok = api.bin_and_sort(proj2, cams2, capacity=20_000_000)
    api.render_forward(proj2, ok, cams2)
    r = ok.read_counters()
    assert not r["overflow"] and r["alive"] > 0 and r["pairs"] > r["pairs1"]
    tight = api.bin_and_sort(proj2, cams2, capacity=r["pairs1"] + 1)
    api.render_forward(proj2, tight, cams2)
    t2 = tight.read_counters()
    assert t2["overflow"] and t2["alive"] > 0 and t2["pairs"] == r["pairs"]


# ------------------------------------------------------------------ a4 forward
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.2, 0.5, 0.9)])
def test_render_forward_parity(dev, case, bg):
    sc, cams = workload(case)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    bins = api.bin_and_sort(proj, cams, capacity=400_000)
    img, T, nc = api.render_forward(proj, bins, cams, bg)
    torch.cuda.synchronize()
    for v, cam in enumerate(cams):
        ref = oracle.render(sc, cam, bg)
        got = to_np(img[v]).transpose(1, 2, 0).reshape(-1, 3)
        check_pixels(got, ref, f"{case} view {v}")
        ok = ref["flag"] == 0
        Tg = to_np(T[v]).reshape(-1)
        assert np.all(np.abs(Tg - ref["T"])[ok] <= 1e-4 * ref["T"][ok] + 1e-7)
        assert Tg.min() >= 1e-4


def test_render_forward_empty_and_culled(dev):
    cam = scenes.Camera(np.eye(3), (0, 0, 4), 40, 40, 20, 15, 40, 30)
    bg = (0.3, 0.6, 0.9)
    for n in (0, 5):
        rng = np.random.default_rng(n)
        # n = 5: all behind the camera
        sc = scenes.Scene(np.tile([[0], [0], [-5.0]], (1, n)), np.full((3, n), -2.0), rng.normal(size=(4, n)),
                          np.zeros(n), np.zeros((1, 3, n)), 0)
        g = api.GaussianTensors.from_scene(sc, dev) if n else api.GaussianTensors.zeros(0, 0, dev)
        proj = api.project_preprocess(g, [cam])
        bins = api.bin_and_sort(proj, [cam], capacity=16)
        img, T, nc = api.render_forward(proj, bins, [cam], bg)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(to_np(img[0]), np.broadcast_to(np.float32(bg)[:, None, None], (3, 30, 40)))
        assert np.all(to_np(T) == 1.0) and np.all(to_np(nc) == 0)


def test_single_tile_image(dev):
    """16x16: one tile, zero tile-key bits, no pair sort pass."""
    w = scenes.tiny(n=300, width=16, height=16)
    cam = scenes.Camera(np.eye(3), (0, 0, 4), 16, 16, 8, 8, 16, 16)
    g = api.GaussianTensors.from_scene(w.scene, dev)
    proj = gpu_preprocess(g, [cam])
    bins = api.bin_and_sort(proj, [cam], capacity=10_000, mode=COMPLETE)
    img, _, _ = api.render_forward(proj, bins, [cam])
    torch.cuda.synchronize()
    _check_bins(bins, proj, [cam], None, False)
    ref = oracle.render(w.scene, cam)
    check_pixels(to_np(img[0]).transpose(1, 2, 0).reshape(-1, 3), ref, "single tile")


# ------------------------------------------------------------------ a5 loss gradient
def test_l1_loss_grad_exact(dev):
    sc, cams = workload("clamp")
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    bins = api.bin_and_sort(proj, cams, capacity=100_000)
    img, _, _ = api.render_forward(proj, bins, cams)
    rng = np.random.default_rng(3)
    tgt_np = rng.uniform(size=img.shape).astype(np.float32)
    tgt_np[0, :, 5, 7] = to_np(img[0, :, 5, 7])      # exact ties give sign 0
    tgt = torch.as_tensor(tgt_np, device=dev)
    loss = torch.zeros(1, device=dev)
    dL = api.l1_loss_grad(img, tgt, bins, cams, loss_sum=loss)
    torch.cuda.synchronize()
    ref_loss, ref_g = oracle.l1_loss_grad(to_np(img[0]), tgt_np[0])
    np.testing.assert_array_equal(to_np(dL[0]), ref_g.astype(np.float32))
    assert abs(float(loss) - ref_loss) <= 1e-5 * ref_loss


@pytest.mark.parametrize("mode", [COMPLETE, api._ffi.BINS_DEPTH_SLICED, api._ffi.BINS_DEPTH_SLICED_LOCAL])
@pytest.mark.parametrize("case,local", [("cloud", False), ("cloud", True), ("local", True)])
def test_forward_with_l1_equals_forward_then_l1(dev, mode, case, local):
    """The forward's own L1 gradient (finished in the second phase for tiles that need
    the second slab) equals the separate L1 call on the stored image, bit for bit."""
    sc, cams, a = _sliced_case(case)
    act = a if local else None
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    bg = (0.1, 0.2, 0.3)
    V, H, W = len(cams), cams[0].height, cams[0].width
    tgt = torch.rand(V, 3, H, W, generator=torch.Generator(device=dev).manual_seed(8), device=dev)
    outs = []
    for fused in (False, True):
        bins = api.bin_and_sort(proj, cams, act, local, capacity=8_000_000, mode=mode)
        state = api.render_state(cams, dev).zero_()   # chunks past a tile's end are not written
        loss = torch.zeros(1, device=dev)
        if fused:
            img, T, nc, dL = api.render_forward_l1(proj, bins, cams, tgt, bg, state=state, loss_sum=loss)
        else:
            img, T, nc = api.render_forward(proj, bins, cams, bg, state=state)
            dL = api.l1_loss_grad(img, tgt, bins, cams, loss_sum=loss)
        torch.cuda.synchronize()
        c = bins.read_counters()
        assert not c["overflow"]
        outs.append((to_np(img), to_np(T), to_np(nc), to_np(dL), float(loss), to_np(state), c))
    (i0, T0, n0, d0, l0, s0, c0), (i1, T1, n1, d1, l1, s1, c1) = outs
    for x, y in ((i0, i1), (T0, T1), (n0, n1), (d0, d1), (s0, s1)):
        np.testing.assert_array_equal(x, y)
    assert abs(l0 - l1) <= 1e-5 * abs(l0) and l0 > 0
    assert np.count_nonzero(d1) > 0
    if mode != COMPLETE and case == "cloud" and not local:
        assert c1["alive"] > 0   # some pixels were finished by the second phase


# ------------------------------------------------------------------ a6, a7 backward
@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("local", [False, True])
def test_render_backward_parity(dev, case, local):
    sc, cams = workload(case)
    n = sc.n
    a = (int(n * 0.75), n) if local else (0, n)
    bg = (0.1, 0.3, 0.2)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    bins = api.bin_and_sort(proj, cams, a, use_mask=local, capacity=400_000)
    state = api.render_state(cams, dev)
    img, T, nc = api.render_forward(proj, bins, cams, bg, state=state)
    rng = np.random.default_rng(21)
    dl_np = rng.normal(size=img.shape).astype(np.float32)
    dl = torch.as_tensor(dl_np, device=dev)
    grads = g.zeros_like()
    api.render_backward(g, proj, bins, cams, bg, a, T, nc, state, dl, grads)
    torch.cuda.synchronize()
    # the reference sees the full image with the same upstream gradient: for the
    # changed Gaussians the local step must give the full-scene gradient
    ref = oracle.gradients(sc, cams, [dl_np[v].astype(np.float64) for v in range(len(cams))], bg)
    worst = check_grads(grads, ref, slice(a[0], a[1]), f"{case} local={local}")
    # rows outside the change set are never written
    for k in api.GaussianTensors.NAMES:
        assert np.all(to_np(getattr(grads, k))[..., :a[0]] == 0)
    print(f"{case} local={local}: worst gradient error / tolerance {worst:.3f}")


def test_render_backward_with_more_items_than_workgroups(dev):
    """A dense scene in one 640x480 view: 1 200 rendered tiles x CLSP_STATE_CHUNKS
    (tile, chunk) items exceed the backward's workgroup count, so workgroups take
    several items each, and tiles reach past their first chunk.  The upstream gradient
    is nonzero at four distinct pixels of every tile, the pixels the oracle evaluates."""
    w = scenes.local_change(n=60_000, n_views=1, width=640, height=480, fx=640.0)
    sc, cams = w.scene, w.cameras
    cam = cams[0]
    n = sc.n
    bg = (0.1, 0.3, 0.2)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    bins = api.bin_and_sort(proj, cams, (0, n), use_mask=False, capacity=20_000_000)
    state = api.render_state(cams, dev)
    img, T, nc = api.render_forward(proj, bins, cams, bg, state=state)
    torch.cuda.synchronize()
    TX, TY = cam.width // 16, cam.height // 16
    hdr = (Path(__file__).resolve().parents[1] / "include" / "clsplat.h").read_text()
    chunk, chunks = (int(re.search(rf"#define {k} (\d+)", hdr).group(1)) for k in ("CLSP_STATE_CHUNK", "CLSP_STATE_CHUNKS"))
    assert bins.read_counters()["tiles"] * chunks > 16_384    # the backward launches at most 16 384 workgroups
    assert int(to_np(nc).max()) > chunk     # some tile's items past its first chunk do work
    rng = np.random.default_rng(8)
    pix = []
    for ty in range(TY):
        for tx in range(TX):
            for o in rng.permutation(256)[:4]:
                pix.append((tx * 16 + o % 16, ty * 16 + o // 16))
    pixels = np.asarray(pix, dtype=np.int32)
    vals = rng.normal(size=(len(pixels), 3)).astype(np.float32)
    dl_np = np.zeros(tuple(img.shape), dtype=np.float32)
    dl_np[0, :, pixels[:, 1], pixels[:, 0]] = vals
    grads = g.zeros_like()
    api.render_backward(g, proj, bins, cams, bg, (0, n), T, nc, state, torch.as_tensor(dl_np, device=dev), grads)
    torch.cuda.synchronize()
    ref = oracle.gradients(sc, cams, [vals.astype(np.float64)], bg, pixels=[pixels])
    worst = check_grads(grads, ref, slice(0, n), "items > workgroups")
    print(f"more items than workgroups: worst gradient error / tolerance {worst:.3f}")


def _deep_scene():
    """Faint, large Gaussians filling a cube seen from 4 units away: every pixel blends
    hundreds of them before its transmittance falls to 1e-4, and tiles list thousands,
    so the compositing state's chunks fill up and merge (twice) and the backward's last
    chunks run deep."""
    rng = np.random.default_rng(21)
    sc = scenes.uniform_cube_scene(rng, 60_000, log_scale_mean=-2.5, log_scale_sd=0.2)
    sc.opacity_logit[:] = np.float32(-3.5)          # opacity 0.029
    cam = scenes.look_at((0.0, 0.0, -4.0), width=128, height=128, fx=128.0, fy=128.0)
    return sc, [cam]


@pytest.mark.parametrize("mode", [COMPLETE, api._ffi.BINS_DEPTH_SLICED, api._ffi.BINS_DEPTH_SLICED_LOCAL])
def test_render_backward_deep_lists(dev, mode):
    """Lists far past CLSP_STATE_CHUNKS x CLSP_STATE_CHUNK entries: the forward merges the
    chunks of the compositing state and doubles their length, and the backward starts
    every chunk of every tile from its stored state; pixels and gradients at eight
    seeded pixels per tile against the reference."""
    sc, cams = _deep_scene()
    cam = cams[0]
    n = sc.n
    bg = (0.1, 0.3, 0.2)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    bins = api.bin_and_sort(proj, cams, None, use_mask=False, capacity=2_000_000, mode=mode)
    state = api.render_state(cams, dev)
    img, T, nc = api.render_forward(proj, bins, cams, bg, state=state)
    torch.cuda.synchronize()
    assert not bins.read_counters()["overflow"]
    hdr = (Path(__file__).resolve().parents[1] / "include" / "clsplat.h").read_text()
    chunk, chunks = (int(re.search(rf"#define {k} (\d+)", hdr).group(1)) for k in ("CLSP_STATE_CHUNK", "CLSP_STATE_CHUNKS"))
    TX, TY = api.tile_grid(cam.width, cam.height)
    ncn = to_np(nc[0]).astype(np.int64)
    per_tile = ncn.reshape(TY, 16, TX, 16).max(axis=(1, 3))
    assert per_tile.max() > 2 * chunks * chunk, per_tile.max()     # two merges of the chunks
    assert (per_tile > chunks * chunk).mean() > 0.25
    rng = np.random.default_rng(9)
    pix = []
    for ty in range(TY):
        for tx in range(TX):
            for o in rng.permutation(256)[:8]:
                pix.append((tx * 16 + o % 16, ty * 16 + o // 16))
    pixels = np.asarray(pix, dtype=np.int32)
    vals = rng.normal(size=(len(pixels), 3)).astype(np.float32)
    dl_np = np.zeros(tuple(img.shape), dtype=np.float32)
    dl_np[0, :, pixels[:, 1], pixels[:, 0]] = vals
    grads = g.zeros_like()
    api.render_backward(g, proj, bins, cams, bg, (0, n), T, nc, state, torch.as_tensor(dl_np, device=dev), grads)
    torch.cuda.synchronize()
    ref = oracle.gradients(sc, cams, [vals.astype(np.float64)], bg, pixels=[pixels])
    got = to_np(img[0])[:, pixels[:, 1], pixels[:, 0]].T
    # each pixel takes thousands of alpha-threshold decisions here (faint Gaussians whose
    # footprints end at alpha = 1/255), so more pixels than usual have one within its
    # float32 error of its threshold; they are excused as everywhere, and counted
    check_pixels(got, oracle.render(sc, cam, bg, pixels=pixels), "deep lists", max_excused=0.03)
    worst = check_grads(grads, ref, slice(0, n), "deep lists")
    print(f"deep lists (max contributor position {per_tile.max()}): worst gradient error / tolerance {worst:.3f}")


def test_capacity_overflow_updates_nothing(dev):
    """A step whose lists ran out of pair capacity writes no gradient, and neither the
    fused backward + Adam nor the Adam call with the overflow flag as its skip flag
    changes parameters or moments."""
    sc, cams = workload("tiny")
    cam = cams[0]
    n = sc.n
    a = (n // 2, n)
    g = api.GaussianTensors.from_scene(sc, dev)
    rng = np.random.default_rng(4)
    m, v = g.zeros_like(), g.zeros_like()
    for t in (m, v):
        for k in api.GaussianTensors.NAMES:
            getattr(t, k).copy_(torch.as_tensor(np.abs(rng.normal(size=tuple(getattr(t, k).shape))).astype(np.float32)
                                                * 1e-3, device=dev))
    g0, m0, v0 = g.clone(), m.clone(), v.clone()
    tgt = torch.rand(1, 3, cam.height, cam.width, generator=torch.Generator(device=dev).manual_seed(1), device=dev)
    proj = gpu_preprocess(g, cams)
    bins = api.bin_and_sort(proj, cams, a, use_mask=True, capacity=64)
    state = api.render_state(cams, dev)
    img, T, nc, dL = api.render_forward_l1(proj, bins, cams, tgt, state=state)
    grads = g.zeros_like()
    api.render_backward(g, proj, bins, cams, (0, 0, 0), a, T, nc, state, dL, grads)
    ws = api.render_backward_workspace(a[1] - a[0], 1, dev)
    api.render_backward_adam(g, proj, bins, cam, (0, 0, 0), a, T, nc, state, dL, m, v, 1, ws=ws)
    api.masked_adam_step(g, grads, m, v, a, 1, skip_flag=bins.counters[1:2])
    torch.cuda.synchronize()
    assert bins.read_counters()["overflow"]
    for k in api.GaussianTensors.NAMES:
        assert not bool(getattr(grads, k).any()), k
        for x, y in ((g, g0), (m, m0), (v, v0)):
            np.testing.assert_array_equal(to_np(getattr(x, k)), to_np(getattr(y, k)))
    assert not bool(ws.any())
    # the same Adam call without the flag does move the moments (zero gradient: decay)
    api.masked_adam_step(g, grads, m, v, a, 1)
    torch.cuda.synchronize()
    assert not np.array_equal(to_np(m.means), to_np(m0.means))


def test_gradients_accumulate(dev):
    """render_backward adds to the gradient buffers.  Two runs sum the same per-pixel
    terms in different orders (float atomics): each term passes through at most 6 DPP
    additions in its wave, 4 LDS atomics of its workgroup and one global atomic per
    tile, so two sums differ by at most 2 (10 + tiles) U32 times the sum of the absolute
    terms (the reference's s, carried through the chain rule), and the accumulation
    itself rounds once more."""
    sc, cams = workload("tiny")
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    bins = api.bin_and_sort(proj, cams, capacity=100_000)
    state = api.render_state(cams, dev)
    img, T, nc = api.render_forward(proj, bins, cams, state=state)
    dl = torch.randn_like(img)
    g1 = g.zeros_like()
    api.render_backward(g, proj, bins, cams, (0, 0, 0), None, T, nc, state, dl, g1)
    g2 = g1.clone()
    api.render_backward(g, proj, bins, cams, (0, 0, 0), None, T, nc, state, dl, g2)
    torch.cuda.synchronize()
    ref = oracle.gradients(sc, cams, [to_np(dl[0]).astype(np.float64)], perturb=0)
    u32 = 2.0 ** -24
    tiles = bins.read_counters()["tiles"]
    for k in api.GaussianTensors.NAMES:
        a, b = to_np(getattr(g1, k)).astype(np.float64), to_np(getattr(g2, k)).astype(np.float64)
        # float32 rounding of the chain rule on the GPU: relative to its magnitude (s)
        tol = 2 * (10 + tiles) * u32 * ref["s"][k] + 1e-5 * ref["s"][k] + 2 * u32 * np.abs(b) + 1e-12
        assert np.all(np.abs(b - 2 * a) <= tol), (k, float((np.abs(b - 2 * a) / tol).max()))
    api.zero_grads(g2, (100, 200))
    torch.cuda.synchronize()
    assert np.all(to_np(g2.means)[:, 100:200] == 0) and np.any(to_np(g2.means)[:, 200:] != 0)


# ------------------------------------------------------------------ exactness of the local step on the GPU
def test_local_step_equals_full_step_on_gpu(dev):
    w = scenes.local_change(n=40_000, n_views=2, width=320, height=180, fx=320.0, radius=0.4)
    sc, cams = w.scene, w.cameras[:1]
    a = (w.active_begin, sc.n)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    out = {}
    for local in (False, True):
        bins = api.bin_and_sort(proj, cams, a if local else None, use_mask=local, capacity=4_000_000)
        state = api.render_state(cams, dev)
        img, T, nc = api.render_forward(proj, bins, cams, state=state)
        tgt = torch.rand_like(img, generator=torch.Generator(device=dev).manual_seed(5))
        dL = api.l1_loss_grad(img, tgt, bins, cams)
        grads = g.zeros_like()
        api.render_backward(g, proj, bins, cams, (0, 0, 0), a if local else None, T, nc, state, dL, grads)
        torch.cuda.synchronize()
        out[local] = (bins, to_np(img), grads)
    pix, tiles = masked_pixels(out[True][0], cams[0])
    assert 0 < len(tiles) < 0.5 * api.tile_grid(320, 180)[0] * api.tile_grid(320, 180)[1]
    # forward on masked tiles: identical lists, identical arithmetic -> identical bits
    li, fi = out[True][1][0], out[False][1][0]
    np.testing.assert_array_equal(li[:, pix[:, 1], pix[:, 0]], fi[:, pix[:, 1], pix[:, 0]])
    for k in api.GaussianTensors.NAMES:
        gl = to_np(getattr(out[True][2], k))[..., a[0]:]
        gf = to_np(getattr(out[False][2], k))[..., a[0]:]
        scale = np.abs(gf).max()
        np.testing.assert_allclose(gl, gf, rtol=1e-4, atol=1e-6 * scale)


@pytest.mark.parametrize("case,local", [("sh3", True), ("sh3", False), ("tiny", True)])
def test_backward_adam_equals_backward_then_adam(dev, case, local):
    """clsp_render_backward_adam equals zero_grads + render_backward + masked_adam_step
    over three steps (so the moments are not trivial) up to the float summation order
    of the raster backward's atomics, which differs between any two runs: nearly every
    element is equal within 1e-5 relative, none is off by more than a few learning
    rates (a wrong component, learning-rate group or missed zero-gradient update would
    move many elements by a learning rate or more)."""
    sc, cams = workload(case)
    cam = cams[0]
    n = sc.n
    a = (n // 2, n) if local else (0, n)
    bg = (0.1, 0.2, 0.3)
    tgt = torch.rand(1, 3, cam.height, cam.width, generator=torch.Generator(device=dev).manual_seed(6), device=dev)
    runs = []
    for fused in (False, True):
        g = api.GaussianTensors.from_scene(sc, dev)
        m, v, grads = g.zeros_like(), g.zeros_like(), g.zeros_like()
        ws = api.render_backward_workspace(a[1] - a[0], 1, dev)   # one workspace for every step
        for step in (1, 2, 3):
            proj = gpu_preprocess(g, [cam])
            bins = api.bin_and_sort(proj, [cam], a if local else None, use_mask=local, capacity=400_000)
            state = api.render_state([cam], dev)
            img, T, nc, dL = api.render_forward_l1(proj, bins, [cam], tgt, bg, state=state)
            if fused:
                api.render_backward_adam(g, proj, bins, cam, bg, a, T, nc, state, dL, m, v, step, ws=ws)
                torch.cuda.synchronize()
                assert not bool(ws.any()), "the fused call leaves its workspace zero"
            else:
                api.zero_grads(grads, a)
                api.render_backward(g, proj, bins, [cam], bg, a, T, nc, state, dL, grads)
                api.masked_adam_step(g, grads, m, v, a, step)
        torch.cuda.synchronize()
        runs.append((g, m, v))
    (g0, m0, v0), (g1, m1, v1) = runs
    moved = 0
    for k in api.GaussianTensors.NAMES:
        for name, x, y, bound in (("params", g0, g1, 6 * max(api.DEFAULT_LR)), ("m", m0, m1, None),
                                  ("v", v0, v1, None)):
            a_, b_ = to_np(getattr(x, k)).astype(np.float64), to_np(getattr(y, k)).astype(np.float64)
            d = np.abs(a_ - b_)
            close = d <= 1e-5 * np.abs(a_) + 1e-6 * (np.abs(a_).max() + 1e-30)
            assert close.mean() >= 0.995, (name, k, float(close.mean()))
            if bound is not None:
                assert d.max() <= bound, (name, k, float(d.max()))
            else:
                assert d.max() <= 0.05 * (np.abs(a_).max() + 1e-30), (name, k, float(d.max()))
        moved += int((to_np(getattr(m1, k)) != 0).sum())
    assert moved > 0


# ------------------------------------------------------------------ a8 masked Adam
@pytest.mark.parametrize("sh_degree", [0, 3])
@pytest.mark.parametrize("with_mask", [False, True])
def test_masked_adam_parity(dev, sh_degree, with_mask):
    rng = np.random.default_rng(sh_degree + 7)
    n, a = 3000, (1200, 3000)
    K = (sh_degree + 1) ** 2
    shapes = {"means": (3, n), "log_scales": (3, n), "quats": (4, n), "opacity_logit": (n,), "sh": (K, 3, n)}
    mk = lambda f: api.GaussianTensors(*[torch.as_tensor(f(s).astype(np.float32), device=dev)
                                         for s in shapes.values()], sh_degree)
    P = mk(lambda s: rng.normal(size=s))
    G = mk(lambda s: rng.normal(size=s) * 0.1)
    M = mk(lambda s: rng.normal(size=s) * 0.01)
    V = mk(lambda s: rng.uniform(size=s) * 1e-3)
    P0, M0, V0 = P.clone(), M.clone(), V.clone()
    row_mask = None
    rows = np.arange(a[0], a[1])
    if with_mask:
        rm = (rng.uniform(size=n) < 0.5).astype(np.uint8)
        row_mask = torch.as_tensor(rm, device=dev)
        rows = rows[rm[a[0]:a[1]] == 1]
    lr = (1e-3, 2e-3, 3e-3, 4e-3, 5e-3, 6e-3)
    step = 7
    # the kernel receives float32 hyper-parameters; the reference gets the same values
    b1, b2, eps = (float(np.float32(x)) for x in (0.9, 0.999, 1e-15))
    lr = tuple(float(np.float32(x)) for x in lr)
    api.masked_adam_step(P, G, M, V, a, step, lr, beta1=b1, beta2=b2, eps=eps, row_mask=row_mask)
    torch.cuda.synchronize()
    names = api.GaussianTensors.NAMES
    np_ = lambda T: {k: to_np(getattr(T, k)).astype(np.float64) for k in names}
    p0, g0, m0, v0 = np_(P0), np_(G), np_(M0), np_(V0)
    e32 = float(np.finfo(np.float32).eps)
    bc1, bc2 = 1 - b1 ** step, 1 - b2 ** step

    def check(key, p, g, m, v, lr_k, got_p, got_m, got_v):
        rP, rM, rV = oracle.adam_step({"x": p}, {"x": g}, {"x": m}, {"x": v}, step, {"x": lr_k}, b1, b2, eps,
                                      rows=rows)
        sl = (Ellipsis, rows)
        # float32 rounding of the moment updates (cancellation in b m + (1 - b) g) ...
        err_m = 4 * e32 * (b1 * np.abs(m[sl]) + (1 - b1) * np.abs(g[sl]))
        err_v = 4 * e32 * (b2 * v[sl] + (1 - b2) * g[sl] ** 2)
        np.testing.assert_array_less(np.abs(got_m[sl] - rM["x"][sl]), err_m + 1e-30)
        np.testing.assert_array_less(np.abs(got_v[sl] - rV["x"][sl]), err_v + 1e-30)
        # ... carried through the step: d/dm and d/dv of lr mhat / (sqrt(vhat) + eps)
        sv = np.sqrt(rV["x"][sl] / bc2)
        step_ = lr_k * (rM["x"][sl] / bc1) / (sv + eps)
        dm = lr_k / bc1 / (sv + eps)
        dv = np.abs(step_) / (sv + eps) / (2 * np.maximum(sv, 1e-30)) / bc2
        ulp = np.spacing(np.abs(rP["x"][sl]).astype(np.float32)).astype(np.float64)
        tol = 1e-6 * np.abs(step_) + dm * err_m + dv * err_v + ulp
        err = np.abs(got_p[sl] - rP["x"][sl])
        assert np.all(err <= tol), (key, float((err / tol).max()))

    gp, gm, gv = np_(P), np_(M), np_(V)
    lrs = {"means": lr[0], "log_scales": lr[1], "quats": lr[2], "opacity_logit": lr[3]}
    for k in names:
        if k != "sh":
            check(k, p0[k], g0[k], m0[k], v0[k], lrs[k], gp[k], gm[k], gv[k])
    # sh: degree-0 rows with lr[4], the rest with lr[5]
    for kk, lr_k in ((slice(0, 1), lr[4]), (slice(1, K), lr[5])):
        if kk.start >= K:
            continue
        check(f"sh{kk}", p0["sh"][kk], g0["sh"][kk], m0["sh"][kk], v0["sh"][kk], lr_k, gp["sh"][kk], gm["sh"][kk],
              gv["sh"][kk])
    # every other row is bit-for-bit untouched
    frozen = np.ones(n, bool)
    frozen[rows] = False
    for T1, T0 in ((P, P0), (M, M0), (V, V0)):
        for k in names:
            np.testing.assert_array_equal(to_np(getattr(T1, k))[..., frozen], to_np(getattr(T0, k))[..., frozen])


@pytest.mark.parametrize("with_mask", [False, True])
def test_masked_adam_clears_gradients_when_asked(dev, with_mask):
    """zero_grads leaves the update bit for bit the same, zeroes every gradient row of
    the active range (masked-out rows too) and no other row."""
    rng = np.random.default_rng(17)
    n, a, sh_degree = 2000, (700, 1900), 1
    K = (sh_degree + 1) ** 2
    shapes = {"means": (3, n), "log_scales": (3, n), "quats": (4, n), "opacity_logit": (n,), "sh": (K, 3, n)}
    mk = lambda f: api.GaussianTensors(*[torch.as_tensor(f(s).astype(np.float32), device=dev)
                                         for s in shapes.values()], sh_degree)
    P, G = mk(lambda s: rng.normal(size=s)), mk(lambda s: rng.normal(size=s) * 0.1)
    M, V = mk(lambda s: rng.normal(size=s) * 0.01), mk(lambda s: rng.uniform(size=s) * 1e-3)
    row_mask = torch.as_tensor((rng.uniform(size=n) < 0.5).astype(np.uint8), device=dev) if with_mask else None
    outs = []
    for zero in (False, True):
        p, g, m, v = P.clone(), G.clone(), M.clone(), V.clone()
        api.masked_adam_step(p, g, m, v, a, 3, row_mask=row_mask, zero_grads=zero)
        outs.append((p, g, m, v))
    torch.cuda.synchronize()
    (p0, g0, m0, v0), (p1, g1, m1, v1) = outs
    inside = np.zeros(n, bool)
    inside[a[0]:a[1]] = True
    for k in api.GaussianTensors.NAMES:
        for X0, X1 in ((p0, p1), (m0, m1), (v0, v1)):
            np.testing.assert_array_equal(to_np(getattr(X1, k)), to_np(getattr(X0, k)))
        got, before = to_np(getattr(g1, k)), to_np(getattr(G, k))
        assert not np.any(got[..., inside])
        np.testing.assert_array_equal(got[..., ~inside], before[..., ~inside])
        np.testing.assert_array_equal(to_np(getattr(g0, k)), before)


# ------------------------------------------------------------------ depth-sliced lists
@pytest.mark.parametrize("case", ["tiny", "ring2", "local", "cloud"])
@pytest.mark.parametrize("local", [False, True])
@pytest.mark.parametrize("sliced_mode", [api._ffi.BINS_DEPTH_SLICED, api._ffi.BINS_DEPTH_SLICED_LOCAL])
def test_depth_sliced_lists_match_complete_lists(dev, case, local, sliced_mode):
    """Every sliced list is a prefix of the complete list (the complete list itself for
    tiles that needed the second slab), and images, transmittance, contributor counts
    are bit-identical; gradients agree up to float32 summation order.  Both ways of
    placing the second slab (sorted, or counted per tile)."""
    sc, cams, a = _sliced_case(case)
    act = a if local else None
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    out = {}
    for mode in (COMPLETE, sliced_mode):
        bins = api.bin_and_sort(proj, cams, act, local, capacity=8_000_000, mode=mode)
        state = api.render_state(cams, dev)
        img, T, nc = api.render_forward(proj, bins, cams, (0.1, 0.2, 0.3), state=state)
        dl = torch.as_tensor(np.random.default_rng(4).normal(size=img.shape).astype(np.float32), device=dev)
        grads = g.zeros_like()
        api.render_backward(g, proj, bins, cams, (0.1, 0.2, 0.3), act, T, nc, state, dl, grads)
        torch.cuda.synchronize()
        c = bins.read_counters()
        assert not c["overflow"]
        out[mode] = (bins, to_np(img), to_np(T), to_np(nc), grads, c)
    cb, ci, cT, cn, cg, cc = out[COMPLETE]
    sb, si, sT, sn, sg, scn = out[sliced_mode]
    np.testing.assert_array_equal(si, ci)
    np.testing.assert_array_equal(sT, cT)
    np.testing.assert_array_equal(sn, cn)
    assert scn["pairs"] <= cc["pairs"] and scn["tiles"] == cc["tiles"]
    vals_c, vals_s = to_np(cb.values).view(np.uint32), to_np(sb.values).view(np.uint32)
    rc = to_np(cb.ranges).view(np.uint32).astype(np.int64)
    r1 = to_np(sb.ranges).view(np.uint32).astype(np.int64)
    r2 = to_np(sb.ranges2).view(np.uint32).astype(np.int64)
    alive = to_np(sb.alive_mask).view(np.uint32)
    TX, TY = api.tile_grid(cams[0].width, cams[0].height)
    T_ = TX * TY
    maxnc = {}
    for gt in to_np(cb.tile_list)[:cc["tiles"]]:
        full = vals_c[rc[gt, 0]:rc[gt, 1]]
        lst = np.concatenate([vals_s[r1[gt, 0]:r1[gt, 1]], vals_s[r2[gt, 0]:r2[gt, 1]]])
        np.testing.assert_array_equal(lst, full[:len(lst)])
        v, t = divmod(int(gt), T_)
        if (alive[v][t // 32] >> (t % 32)) & 1:
            assert len(lst) == len(full)
    # the sliced lists reach every pixel's last contributor
    for v in range(len(cams)):
        ncv = cn[v]
        for gt in to_np(cb.tile_list)[:cc["tiles"]]:
            vv, t = divmod(int(gt), T_)
            if vv != v:
                continue
            ty, tx = divmod(t, TX)
            m = int(ncv[ty * 16:(ty + 1) * 16, tx * 16:(tx + 1) * 16].max(initial=0))
            assert (r1[gt, 1] - r1[gt, 0]) + (r2[gt, 1] - r2[gt, 0]) >= m
    rows = slice(a[0], a[1]) if local else slice(0, sc.n)
    for k in api.GaussianTensors.NAMES:
        x = to_np(getattr(sg, k))[..., rows].astype(np.float64)
        y = to_np(getattr(cg, k))[..., rows].astype(np.float64)
        scale = np.sqrt((y ** 2).mean()) + 1e-30
        assert np.abs(x - y).max() <= 1e-4 * np.abs(y).max() + 1e-3 * scale, k
    if case == "local":
        assert scn["pairs"] < cc["pairs"]           # the dense local scene terminates early
    if case == "cloud" and not local:
        assert scn["alive"] > 0                     # some tiles needed the second slab

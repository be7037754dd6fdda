"""Lists of local optimisation built from a stored depth order of the unchanged rows
(clsp_frozen_order + clsp_bin_and_sort_frozen): bit for bit the lists of the reference
on the small cases, and the lists of clsp_bin_and_sort (use_mask, active = [a0, n)) on
depth-sliced and full-size cases, with the same forward images (Supp. "Local
Optimization Kernel", item 1: the projection of the unchanged Gaussians, and so their
depth order, is reused)."""
import numpy as np
import pytest
import torch

import scenes
from gpu_helpers import gpu_preprocess, to_np
from paper_2506_21117_amd import _ffi, api
from test_gpu_parity import CASES, _check_bins, _sliced_case, workload

pytestmark = pytest.mark.gpu
COMPLETE = _ffi.BINS_COMPLETE


def _frozen_bins(proj, cams, a0, **kw):
    order = api.frozen_order(proj, cams, a0)
    return api.bin_and_sort_frozen(proj, cams, order, **kw), order


def _same_lists(a, b):
    ca, cb = a.read_counters(), b.read_counters()
    assert ca == cb
    P = ca["written"]
    np.testing.assert_array_equal(to_np(a.values)[:P], to_np(b.values)[:P])
    np.testing.assert_array_equal(to_np(a.keys)[:P], to_np(b.keys)[:P])
    for k in ("ranges", "ranges2", "tile_mask", "alive_mask"):
        np.testing.assert_array_equal(to_np(getattr(a, k)), to_np(getattr(b, k)), err_msg=k)
    np.testing.assert_array_equal(to_np(a.tile_list)[:ca["tiles"]], to_np(b.tile_list)[:cb["tiles"]])
    return ca


@pytest.mark.parametrize("case", CASES)
def test_frozen_order_lists_bit_exact(dev, case):
    sc, cams = workload(case)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    active = (int(sc.n * 0.8), sc.n)
    bins, _ = _frozen_bins(proj, cams, active[0], capacity=200_000, mode=COMPLETE)
    torch.cuda.synchronize()
    assert _check_bins(bins, proj, cams, active, True) > 0


def test_frozen_order_many_tile_bits(dev):
    """3600 tiles per view, two views: entries of both views in one stored order."""
    w = scenes.full_scene(n=4000, n_views=2, res=960, fx=1320.0)
    cams = [scenes.Camera(c.R, c.t, 1280, 1280, 640, 360, 1280, 720) for c in w.cameras]
    g = api.GaussianTensors.from_scene(w.scene, dev)
    proj = gpu_preprocess(g, cams)
    bins, _ = _frozen_bins(proj, cams, 3000, capacity=2_000_000, mode=COMPLETE)
    torch.cuda.synchronize()
    _check_bins(bins, proj, cams, (3000, 4000), True)


@pytest.mark.parametrize("a0_frac", [0.0, 1.0, 0.999])
def test_frozen_order_edge_cases(dev, a0_frac):
    """No unchanged rows (every entry sorted), no changed rows (empty mask: no tiles, no
    pairs), a change set of a handful of rows."""
    sc, cams = workload("ring2")
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    a0 = int(round(sc.n * a0_frac))
    bins, _ = _frozen_bins(proj, cams, a0, capacity=400_000, mode=COMPLETE)
    torch.cuda.synchronize()
    P = _check_bins(bins, proj, cams, (a0, sc.n), True)
    plain = api.bin_and_sort(proj, cams, (a0, sc.n), True, capacity=400_000, mode=COMPLETE)
    torch.cuda.synchronize()
    assert _same_lists(bins, plain)["pairs"] == P
    if a0 == sc.n:
        assert P == 0 and bins.read_counters()["tiles"] == 0


@pytest.mark.parametrize("name", ["local", "cloud"])
def test_frozen_order_depth_sliced_same_render(dev, name):
    """Depth-sliced lists (both slabs) and the forward over them equal those of the full
    sort, bit for bit; the stored order is reused for a second binning after the change
    set moved."""
    sc, cams, active = _sliced_case(name)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    order = api.frozen_order(proj, cams, active[0])
    for it in range(2):
        if it == 1:
            gen = torch.Generator(device=dev).manual_seed(11)
            g.means[:, active[0]:] += 0.01 * torch.randn(g.means[:, active[0]:].shape, generator=gen, device=dev)
            proj = gpu_preprocess(g, cams)
        fb = api.bin_and_sort_frozen(proj, cams, order, capacity=20_000_000)
        pb = api.bin_and_sort(proj, cams, active, True, capacity=20_000_000)
        img_f, T_f, nc_f = api.render_forward(proj, fb, cams)
        img_p, T_p, nc_p = api.render_forward(proj, pb, cams)
        torch.cuda.synchronize()
        c = _same_lists(fb, pb)
        assert not c["overflow"] and c["tiles"] > 0
        for a, b in ((img_f, img_p), (T_f, T_p), (nc_f, nc_p)):
            np.testing.assert_array_equal(to_np(a), to_np(b))
    if name == "cloud":
        assert c["alive"] > 0


@pytest.mark.parametrize("center", [(0.0, 0.0, 0.0), (0.0, 0.0, 1.0)])
def test_frozen_order_full_size_same_lists(dev, center):
    """The benchmark's local step (10^6 Gaussians, 1280x720, the change ball occluded or
    visible), one view: the same lists and render as the full sort."""
    w = scenes.local_change(center=center)
    sc, cam = w.scene, [w.cameras[3]]
    a0 = w.active_begin
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cam)
    print(f"full-size frozen order: center {center}, a0 {a0}, n {sc.n}", flush=True)
    fb, _ = _frozen_bins(proj, cam, a0, capacity=40_000_000)
    pb = api.bin_and_sort(proj, cam, (a0, sc.n), True, capacity=40_000_000)
    img_f, T_f, _ = api.render_forward(proj, fb, cam)
    img_p, T_p, _ = api.render_forward(proj, pb, cam)
    torch.cuda.synchronize()
    c = _same_lists(fb, pb)
    assert not c["overflow"] and c["pairs"] > 100_000 and c["entries"] > 100_000
    np.testing.assert_array_equal(to_np(img_f), to_np(img_p))
    np.testing.assert_array_equal(to_np(T_f), to_np(T_p))


def test_optimizer_local_steps_with_and_without_frozen_order(dev):
    """Local steps over several views, two optimisers in lockstep: with the stored orders
    every step's lists equal those of the full sort, bit for bit.  After the first step
    the Adam moments (0.1 x the gradient) agree up to the order of the backward's float
    additions (atomics and wave reductions): 1e-4 relative, with a floor of 1e-6 of the
    largest moment for terms that cancel to rounding residue.  (Later
    steps are not compared element by element: Adam turns the sign of such a residue into
    a step of size lr.)"""
    from paper_2506_21117_amd.optim import SplatOptimizer
    w = scenes.local_change(n=40_000, n_views=3, width=320, height=180, fx=320.0, center=(0.0, 0.0, 1.0))
    sc, cams = w.scene, w.cameras
    a0, n = w.active_begin, sc.n
    tg = torch.rand(3, 3, 180, 320, generator=torch.Generator(device=dev).manual_seed(5), device=dev)
    opts = [SplatOptimizer(api.GaussianTensors.from_scene(sc, dev), cams, tg, active=(a0, n), local=True,
                           frozen_order=f) for f in (True, False)]
    compared = False
    for k in range(7):
        for o in opts:
            o.step(k % 3)
        torch.cuda.synchronize()
        c = _same_lists(opts[0].bins, opts[1].bins)
        assert c["pairs"] > 0
        # the first step with gradients (before it nothing moved: zero gradients leave the
        # moments and the parameters as they were)
        m0 = {name: [to_np(getattr(o.m, name))[..., a0:].astype(np.float64) for o in opts]
              for name in api.GaussianTensors.NAMES}
        if not compared and sum(int(np.count_nonzero(x[0])) for x in m0.values()) > 1000:
            # the change set is isotropic: its quaternion gradients are zero in exact
            # arithmetic and rounding residue on both sides, so the floor is taken from the
            # step's largest moment over all parameters
            floor = 1e-6 * max(np.abs(x).max() for pair in m0.values() for x in pair)
            for name, (a, b) in m0.items():
                np.testing.assert_allclose(a, b, rtol=1e-4, atol=floor, err_msg=name)
            compared = True
    assert compared
    assert not any(o.overflowed() for o in opts)
    assert bool(opts[0]._frozen_orders) and not opts[1]._frozen_orders
    assert not np.array_equal(to_np(opts[0].params.means)[:, a0:], sc.means[:, a0:])


@pytest.mark.parametrize("a0", [0, 5000, 39_000])
def test_frozen_order_change_set_sizes(dev, a0):
    """Change sets of 80 000, 70 000 and 2 000 entries (several sort blocks, each with
    several chunks, and one): the same lists as the full sort, both slabs."""
    sc, cams, _ = _sliced_case("cloud")
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    fb, _ = _frozen_bins(proj, cams, a0, capacity=40_000_000)
    pb = api.bin_and_sort(proj, cams, (a0, sc.n), True, capacity=40_000_000)
    img_f, _, _ = api.render_forward(proj, fb, cams)
    img_p, _, _ = api.render_forward(proj, pb, cams)
    torch.cuda.synchronize()
    c = _same_lists(fb, pb)
    assert not c["overflow"] and c["entries"] > 0
    np.testing.assert_array_equal(to_np(img_f), to_np(img_p))

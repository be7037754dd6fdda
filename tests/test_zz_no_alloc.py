"""The allocation-free backward (clsp_render_backward_noalloc, its screen-space
gradients in the library's static per-GPU scratch) against clsp_render_backward (the
same kernels on a caller workspace) and against the oracle, on two calls in a row, the
second with a smaller change set: the scratch keeps the first call's contents, so a
missing clear would show in the second."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_helpers import check_grads, gpu_preprocess, to_np
from paper_2506_21117_amd import api

pytestmark = pytest.mark.gpu


def _ring2():
    w = scenes.full_scene(n=3000, n_views=2, res=96, fx=132.0)
    return w.scene, w.cameras


def _tiny():
    w = scenes.tiny()
    return w.scene, w.cameras


def _one_call(dev, sc, cams, active, local, seed):
    n = sc.n
    bg = (0.1, 0.3, 0.2)
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, cams)
    bins = api.bin_and_sort(proj, cams, active, use_mask=local, capacity=400_000)
    state = api.render_state(cams, dev)
    img, T, nc = api.render_forward(proj, bins, cams, bg, state=state)
    dl_np = np.random.default_rng(seed).normal(size=tuple(img.shape)).astype(np.float32)
    dl = torch.as_tensor(dl_np, device=dev)
    with_ws = g.zeros_like()
    api.render_backward(g, proj, bins, cams, bg, active, T, nc, state, dl, with_ws)
    no_ws = g.zeros_like()
    api.render_backward_noalloc(g, proj, bins, cams, bg, active, T, nc, state, dl, no_ws)
    torch.cuda.synchronize()
    assert not bins.read_counters()["overflow"]
    tiles = bins.read_counters()["tiles"]
    ref = oracle.gradients(sc, cams, [dl_np[v].astype(np.float64) for v in range(len(cams))], bg)
    a0, a1 = active
    worst = check_grads(no_ws, ref, slice(a0, a1), f"noalloc n={n} views={len(cams)}")
    # against the workspace call: the same per-pixel terms summed in another order by
    # the float atomics (at most 6 DPP + 4 LDS additions and one global atomic per tile
    # per term), so the two differ by at most 2 (10 + tiles) u32 times the sum of the
    # absolute terms (the oracle's s), plus one rounding of each result
    u32 = 2.0 ** -24
    for k in api.GaussianTensors.NAMES:
        a = to_np(getattr(with_ws, k)).astype(np.float64)
        b = to_np(getattr(no_ws, k)).astype(np.float64)
        s = ref["s"][k]
        tol = 2 * (10 + tiles) * u32 * s + 1e-5 * s + 2 * u32 * np.abs(a) + 1e-12
        assert np.all(np.abs(b - a) <= tol), (k, float((np.abs(b - a) / tol).max()))
        assert np.all(b[..., :a0] == 0) and np.all(b[..., a1:] == 0), k   # rows outside the change set
    return worst


def test_noalloc_backward_equals_workspace_backward_twice(dev):
    sc, cams = _ring2()
    w1 = _one_call(dev, sc, cams, (0, sc.n), False, 31)            # 3 000 rows x 2 views
    sc2, cams2 = _tiny()
    w2 = _one_call(dev, sc2, cams2, (1500, sc2.n), True, 32)       # 500 rows x 1 view
    print(f"noalloc: worst gradient error / tolerance {w1:.3f}, then {w2:.3f}")

"""The L1 + D-SSIM loss gradient on the GPU (clsp_l1_dssim_loss_grad) against the CPU
reference, and its local form: on the masked tiles of a local step, with the unchanged
Gaussians' render supplying the pixels around them, it equals the full-image gradient
bit for bit (the paper's loss, Supp. "Implementation Details"; exactness of the local
kernel, Sec. 3.3 "Local Optimization Kernel").

Bar against the reference: both evaluate the window sums and SSIM partials in double
(in different orders, ~1e-15 of the terms' sizes), the GPU rounds the gradient to float
once: |g - o| <= u32 |o| + 1e-9 / (3 H W)."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_helpers import gpu_preprocess, masked_pixels, to_np
from paper_2506_21117_amd import api

pytestmark = pytest.mark.gpu
U32 = 2.0 ** -24


def _full_bins(dev, w, h, views=1):
    """Lists of every tile (only the tile list, mask and counters are read)."""
    sc = scenes.tiny(n=50, width=w, height=h).scene
    cams = [scenes.Camera(np.eye(3), (0, 0, 4), w, w, w / 2, h / 2, w, h)] * views
    g = api.GaussianTensors.from_scene(sc, dev)
    return api.bin_and_sort(gpu_preprocess(g, cams), cams, capacity=1 << 16), cams


@pytest.mark.parametrize("w,h,views", [(64, 48, 1), (100, 37, 2), (16, 16, 1), (5, 3, 1)])
def test_l1_dssim_gradient_parity(dev, w, h, views):
    bins, cams = _full_bins(dev, w, h, views)
    rng = np.random.default_rng(w + h)
    img = rng.random((views, 3, h, w)).astype(np.float32)
    tgt = rng.random((views, 3, h, w)).astype(np.float32)
    img[:, :, : h // 2, : w // 3] = tgt[:, :, : h // 2, : w // 3]     # a region where x = y (sign 0, SSIM near 1)
    img[0, 1, :, :] = 0.5                                              # a flat channel (small variances)
    loss = torch.zeros(1, device=dev)
    dl = api.l1_dssim_loss_grad(torch.as_tensor(img, device=dev), torch.as_tensor(tgt, device=dev), bins, cams,
                                loss_sum=loss)
    torch.cuda.synchronize()
    got = to_np(dl).astype(np.float64)
    total = 0.0
    # the C-ABI takes lambda as a float: the reference takes the same value (where the L1
    # and SSIM parts cancel, 0.2 and float(0.2) differ visibly)
    lam = float(np.float32(api.LAMBDA_DSSIM))
    for v in range(views):
        ref_loss, ref = oracle.l1_dssim_loss_grad(img[v], tgt[v], lam=lam)
        total += ref_loss
        err = np.abs(got[v] - ref)
        tol = U32 * np.abs(ref) + 1e-9 / (3 * w * h)
        assert np.all(err <= tol), float((err / tol).max())
    assert abs(float(loss.item()) - total) <= 1e-5 * total


def test_local_l1_dssim_equals_full_on_masked_tiles(dev):
    """A local step's render (masked tiles only; the rest of the image buffer holds
    garbage) plus the render of the unchanged Gaussians gives, on the masked tiles, the
    gradient of the full render bit for bit."""
    w = scenes.local_change(n=40_000, n_views=2, width=320, height=180, fx=320.0, center=(0.0, 0.0, 1.0))
    sc, cam = w.scene, w.cameras[1]
    a0, n = w.active_begin, sc.n
    g = api.GaussianTensors.from_scene(sc, dev)
    proj = gpu_preprocess(g, [cam])
    full = api.bin_and_sort(proj, [cam], capacity=4_000_000)
    img_full, _, _ = api.render_forward(proj, full, [cam])
    local = api.bin_and_sort(proj, [cam], (a0, n), use_mask=True, capacity=4_000_000)
    img_local = torch.rand_like(img_full) * 7.0
    api.render_forward(proj, local, [cam], image=img_local)
    # the unchanged Gaussians alone: the first a0 rows
    frozen_g = api.GaussianTensors(*[getattr(g, k)[..., :a0].contiguous() for k in api.GaussianTensors.NAMES],
                                   g.sh_degree)
    pf = gpu_preprocess(frozen_g, [cam])
    bf = api.bin_and_sort(pf, [cam], capacity=4_000_000)
    img_frozen, _, _ = api.render_forward(pf, bf, [cam])
    tgt = torch.rand_like(img_full)
    d_full = api.l1_dssim_loss_grad(img_full, tgt, full, [cam])
    d_local = api.l1_dssim_loss_grad(img_local, tgt, local, [cam], frozen=img_frozen)
    torch.cuda.synchronize()
    for b in (full, local, bf):
        assert not b.read_counters()["overflow"]
    pix, tiles = masked_pixels(local, cam)
    assert 0 < len(tiles) < 0.5 * api.tile_grid(cam.width, cam.height)[0] * api.tile_grid(cam.width, cam.height)[1]
    a = to_np(d_full[0])[:, pix[:, 1], pix[:, 0]]
    b = to_np(d_local[0])[:, pix[:, 1], pix[:, 0]]
    np.testing.assert_array_equal(a, b)
    assert np.count_nonzero(a) > 0.9 * a.size


def test_optimizer_local_step_with_l1_dssim_gets_the_full_gradient(dev):
    """One local step of the optimiser with the L1 + D-SSIM loss: the first Adam moment
    of the change set is (1 - beta1) times the gradient of a full-scene render with the
    same loss (the same per-pixel terms summed in another atomic order)."""
    from paper_2506_21117_amd.optim import SplatOptimizer
    w = scenes.local_change(n=40_000, n_views=2, width=320, height=180, fx=320.0, center=(0.0, 0.0, 1.0))
    sc, cams = w.scene, w.cameras
    a0, n = w.active_begin, sc.n
    tg = torch.rand(2, 3, 180, 320, generator=torch.Generator(device=dev).manual_seed(9), device=dev)
    g = api.GaussianTensors.from_scene(sc, dev)
    ref_g = g.clone()
    opt = SplatOptimizer(g, cams, tg, active=(a0, n), local=True, loss="l1_dssim")
    opt.step(1)
    # full render of the same view with the same loss, every row active
    cam = [cams[1]]
    proj = gpu_preprocess(ref_g, cam)
    bins = api.bin_and_sort(proj, cam, capacity=4_000_000)
    state = api.render_state(cam, dev)
    img, T, nc = api.render_forward(proj, bins, cam, state=state)
    dL = api.l1_dssim_loss_grad(img, tg[1:2].contiguous(), bins, cam)
    grads = ref_g.zeros_like()
    api.render_backward(ref_g, proj, bins, cam, (0, 0, 0), None, T, nc, state, dL, grads)
    torch.cuda.synchronize()
    assert not opt.overflowed()
    # the re-initialised change set is isotropic: its quaternion gradients are zero in
    # exact arithmetic and rounding residue on both sides, so the absolute floor is taken
    # from the step's largest gradient over all parameters
    full = {k: to_np(getattr(grads, k))[..., a0:].astype(np.float64) for k in api.GaussianTensors.NAMES}
    floor = 1e-6 * max(np.abs(x).max() for x in full.values())
    moved = 0
    for k in api.GaussianTensors.NAMES:
        m = to_np(getattr(opt.m, k))[..., a0:].astype(np.float64) / 0.1
        np.testing.assert_allclose(m, full[k], rtol=1e-4, atol=floor, err_msg=k)
        moved += int(np.count_nonzero(full[k]))
    assert moved > 1000

"""Pins of the L1 + D-SSIM loss of the CPU reference (the 3D Gaussian Splatting default
loss the paper trains with, Supp. "Implementation Details"): the window, SSIM closed
forms, and the analytic gradient against float64 central differences."""
import numpy as np

import oracle


def test_window_is_the_normalised_gaussian():
    w = oracle.ssim_window()
    assert w.shape == (11, 11) and abs(w.sum() - 1) < 1e-15
    np.testing.assert_allclose(w, w.T, rtol=0, atol=0)
    assert abs(w[5, 6] / w[5, 5] - np.exp(-1 / (2 * 1.5 ** 2))) < 1e-15
    assert abs(w[5, 10] / w[5, 5] - np.exp(-25 / (2 * 1.5 ** 2))) < 1e-15


def test_ssim_of_identical_images_is_one_and_stationary():
    x = np.random.default_rng(0).random((3, 20, 17))
    s = oracle.ssim_map(x, x)
    np.testing.assert_allclose(s, 1.0, atol=1e-12)
    loss, g = oracle.l1_dssim_loss_grad(x, x)
    assert abs(loss) < 1e-12 and np.abs(g).max() < 1e-12


def test_ssim_of_constant_images_in_the_interior():
    a, b = 0.3, 0.7
    s = oracle.ssim_map(np.full((1, 30, 30), a), np.full((1, 30, 30), b))
    want = (2 * a * b + 0.01 ** 2) / (a * a + b * b + 0.01 ** 2)
    np.testing.assert_allclose(s[0, 5:25, 5:25], want, rtol=1e-12)
    assert np.all(np.abs(s[0, 0, :] - want) > 1e-6)       # the zero padding changes the border


def test_gradient_against_central_differences():
    rng = np.random.default_rng(1)
    x, y = rng.random((3, 12, 13)), rng.random((3, 12, 13))
    loss, g = oracle.l1_dssim_loss_grad(x, y)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 5, 6), (2, 11, 12), (0, 6, 0), (1, 0, 7), (2, 3, 9)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (oracle.l1_dssim_loss_grad(xp, y)[0] - oracle.l1_dssim_loss_grad(xm, y)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-7 * abs(g[idx]) + 1e-10, (idx, fd, g[idx])
    # lambda = 1: the D-SSIM part alone; lambda = 0: the L1 gradient sign(x - y)/n
    l0, g0 = oracle.l1_dssim_loss_grad(x, y, lam=0.0)
    np.testing.assert_allclose(g0, np.sign(x - y) / x.size, rtol=1e-15)
    assert abs(l0 - np.abs(x - y).mean()) < 1e-15

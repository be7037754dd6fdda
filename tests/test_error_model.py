"""The float32 error term of the gradient comparison.

The oracle bounds, per Gaussian and view, how far a float32 evaluation of the
projected quantities (u, v, the conic, the colour) can be from their exact values
(``oracle.error_bounds``), and the gradient bar moves every Gaussian by those amounts
with random signs and measures how far the gradient moves (``oracle.gradients``,
key ``"e"``).  These tests pin the bounds to an independent float32 evaluation of the
same definitions (plain numpy float32 arithmetic, correctly rounded operations in an
order of its own) and check that the resulting bar still detects small gradient
errors.
"""
import numpy as np
import pytest

import oracle
import scenes

F = np.float32
SH_C = [0.28209479177387814, 0.4886025119029199, 1.0925484305920792, 0.31539156525252005, 0.5462742152960396,
        0.5900435899266435, 2.890611442640554, 0.4570457994644658, 0.3731763325901154, 1.445305721320277]


def f32_projection(sc, cam):
    """u, v, conic (A, B, C) and colour [3, N] in numpy float32, from the definitions:
    p = R mu + t, u = fx X/Z + cx; Sigma = R(q) diag(s^2) R(q)^T; cov2 = J Rcam Sigma
    Rcam^T J^T + 0.3 I with the lateral ratios clamped to 1.3 of the half-image tangent;
    colour = max(0, 0.5 + sum_k f_k Y_k(dir))."""
    mu = sc.means.astype(F)
    R = np.asarray(cam.R, F)
    t = np.asarray(cam.t, F)
    X, Y, Z = R @ mu + t[:, None]
    u = F(cam.fx) * (X / Z) + F(cam.cx)
    v = F(cam.fy) * (Y / Z) + F(cam.cy)
    q = sc.quats.astype(F)
    q = q / np.sqrt((q * q).sum(0))
    w, x, y, z = q
    one, two = F(1), F(2)
    Rq = np.stack([one - two * (y * y + z * z), two * (x * y - w * z), two * (x * z + w * y),
                   two * (x * y + w * z), one - two * (x * x + z * z), two * (y * z - w * x),
                   two * (x * z - w * y), two * (y * z + w * x), one - two * (x * x + y * y)]).reshape(3, 3, -1)
    s = np.exp(sc.log_scales.astype(F))
    Sig = np.einsum("ikn,kn,jkn->ijn", Rq, s * s, Rq).astype(F)
    limx = F(1.3 * 0.5 * cam.width / cam.fx)
    limy = F(1.3 * 0.5 * cam.height / cam.fy)
    tx = np.clip(X / Z, -limx, limx)
    ty = np.clip(Y / Z, -limy, limy)
    J = np.zeros((2, 3, X.size), F)
    J[0, 0] = F(cam.fx) / Z
    J[0, 2] = -F(cam.fx) * tx / Z
    J[1, 1] = F(cam.fy) / Z
    J[1, 2] = -F(cam.fy) * ty / Z
    M = np.einsum("akn,kb->abn", J, R).astype(F)
    cov = np.einsum("akn,kln,bln->abn", M, Sig, M).astype(F)
    a, b, c = cov[0, 0] + F(0.3), cov[0, 1], cov[1, 1] + F(0.3)
    det = a * c - b * b
    K = np.stack([c / det, -b / det, a / det])
    # colour
    cp = (-(np.asarray(cam.R, np.float64).T @ np.asarray(cam.t, np.float64))).astype(F)
    d = mu - cp[:, None]
    d = d / np.sqrt((d * d).sum(0))
    x, y, z = d
    C = [F(c_) for c_ in SH_C]
    Yb = [C[0] + 0 * x, C[1] * y, C[1] * z, C[1] * x, C[2] * x * y, C[2] * y * z, C[3] * (F(3) * z * z - F(1)),
          C[2] * x * z, C[4] * (x * x - y * y), C[5] * y * (F(3) * x * x - y * y), C[6] * x * y * z,
          C[7] * y * (F(5) * z * z - F(1)), C[8] * z * (F(5) * z * z - F(3)), C[7] * x * (F(5) * z * z - F(1)),
          C[9] * z * (x * x - y * y), C[5] * x * (x * x - F(3) * y * y)]
    col = np.zeros((3, sc.n), F) + F(0.5)
    sh = sc.sh.astype(F)
    for k in range((sc.sh_degree + 1) ** 2):
        col = col + sh[k] * Yb[k]
    return u, v, K, np.maximum(col, F(0))


WORKLOADS = {
    "tiny": lambda: scenes.tiny(),
    "sh3": lambda: scenes.fd_scene(n=500, res=64),
    "local": lambda: scenes.local_change(n=60_000, n_views=2, width=1280, height=720, fx=1280.0),
    "full": lambda: scenes.full_scene(n=20_000, n_views=2, res=800, fx=1100.0),
}


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_float32_projection_stays_within_the_error_bounds(orc, name):
    w = WORKLOADS[name]()
    for cam in w.cameras[:2]:
        ref = orc.preprocess(w.scene, cam)
        eb = orc.error_bounds(w.scene, cam)
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            u, v, K, col = f32_projection(w.scene, cam)
        vis = ref["visible"] & ((ref["flags"] & (orc.F_CLAMPX | orc.F_CLAMPY | orc.F_NEAR)) == 0)
        assert vis.sum() > 0.3 * w.scene.n
        ratios = {
            "u": np.abs(u - ref["u"])[vis] / eb["u"][vis],
            "v": np.abs(v - ref["v"])[vis] / eb["v"][vis],
            "K": np.max(np.abs(K - np.stack([ref["A"], ref["B"], ref["C"]])), 0)[vis] / eb["K"][vis],
            "rgb": (np.abs(col.T - np.stack([ref["r"], ref["g"], ref["b"]], 1))[vis] / eb["rgb"][vis]),
        }
        for k, r in ratios.items():
            # a bound, with room for an evaluation in another order, but not vacuous
            assert r.max() < 0.7, (k, float(r.max()))
            assert np.median(r) > 1e-3, (k, float(np.median(r)))


@pytest.mark.parametrize("name", ["tiny", "sh3"])
def test_gradient_bar_detects_two_percent_errors(orc, name):
    """With the float32 terms included, a 2% error of a gradient entry exceeds the bar
    for at least 90% of the entries, and at least 80% of the quaternion entries: the
    quaternion gradient of a nearly isotropic Gaussian (these scenes draw each axis'
    log-scale from N(-3, 0.5)) is a small difference of large terms, so the rounding
    allowance s, the size of the terms a float32 evaluation cancels, is large against
    its value (median s/|g| ~ 240 here against ~8 for the means)."""
    w = WORKLOADS[name]()
    cam = w.cameras[0]
    dl = np.random.default_rng(1).normal(size=(3, cam.height, cam.width))
    ref = orc.gradients(w.scene, [cam], [dl], (0.1, 0.3, 0.2))
    for k in ("means", "log_scales", "quats", "opacity_logit", "sh"):
        o, s, e = ref[k], ref["s"][k], ref["e"][k]
        nz = s > 0
        tol = 1e-3 * np.abs(o) + 1e-5 * s + e
        assert (tol[nz] < 0.02 * np.abs(o[nz])).mean() >= (0.8 if k == "quats" else 0.9), k


def test_rounding_allowance_covers_cancelled_quaternion_terms(orc):
    """A Gaussian with three equal scales has an exactly zero quaternion gradient, but
    its float32 evaluation cancels terms of the size of the other gradients: the
    rounding allowance s is positive there and of that size, not zero."""
    w = scenes.tiny(n=300)
    sc = w.scene
    sc.log_scales[:] = sc.log_scales[:1]          # equal scales per Gaussian
    cam = w.cameras[0]
    dl = np.random.default_rng(2).normal(size=(3, cam.height, cam.width))
    ref = orc.gradients(sc, [cam], [dl], perturb=0)
    hit = ref["s"]["means"].sum(0) > 0
    assert hit.sum() > 50
    assert np.all(np.abs(ref["quats"][:, hit]) <= 1e-12 * ref["s"]["quats"][:, hit] + 1e-300)
    assert np.all(ref["s"]["quats"][1:, hit].max(0) > 1e-3 * np.abs(ref["means"][:, hit]).max(0))


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_float32_exponent_stays_within_its_bound(orc, name):
    """The band in which the oracle flags a pixel's alpha decisions as near a threshold
    (a float32 evaluation may take them either way) is its bound on the float32 error
    of the exponent -d^T K d / 2: the centre's bounds times |K d|, the covariance's
    times |K d|^2, the inversion's rounding times |exponent|, and the quadratic form's
    own rounding.  An independent float32 evaluation of the exponent at pixel centres
    on the alpha = 1/255 ellipse, in eight directions, stays inside it."""
    w = WORKLOADS[name]()
    cam = w.cameras[0]
    ref = orc.preprocess(w.scene, cam)
    eb = orc.error_bounds(w.scene, cam)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        u32, v32, K32, _ = f32_projection(w.scene, cam)
    vis = ref["visible"] & ((ref["flags"] & (orc.F_CLAMPX | orc.F_CLAMPY | orc.F_NEAR)) == 0)
    idx = np.nonzero(vis)[0]
    idx = np.random.default_rng(7).choice(idx, size=min(4000, len(idx)), replace=False)
    A, B, C = ref["A"][idx], ref["B"][idx], ref["C"][idx]
    kap = 2.0 * np.log(255.0 * ref["opacity"][idx])
    u32 = u32.astype(np.float64)[idx].astype(F)
    v32 = v32.astype(np.float64)[idx].astype(F)
    K32 = K32[:, idx]
    ratios = []
    for th in np.arange(8) * np.pi / 8:
        ex, ey = np.cos(th), np.sin(th)
        r = np.sqrt(kap / (A * ex * ex + 2 * B * ex * ey + C * ey * ey))
        px = np.floor(ref["u"][idx] + r * ex) + 0.5
        py = np.floor(ref["v"][idx] + r * ey) + 0.5
        dx, dy = px - ref["u"][idx], py - ref["v"][idx]
        q = A * dx * dx + 2 * B * dx * dy + C * dy * dy
        qabs = np.abs(A * dx * dx) + 2 * np.abs(B * dx * dy) + np.abs(C * dy * dy)
        dx32, dy32 = px.astype(F) - u32, py.astype(F) - v32
        q32 = K32[0] * dx32 * dx32 + F(2) * K32[1] * dx32 * dy32 + K32[2] * dy32 * dy32
        Ku, Kv = A * dx + B * dy, B * dx + C * dy
        bound = (np.abs(Ku) * eb["u"][idx] + np.abs(Kv) * eb["v"][idx] + (Ku * Ku + Kv * Kv) * eb["cov"][idx]
                 + 0.5 * q * eb["det"][idx] + 4 * 2.0 ** -24 * qabs)
        ratios.append(np.abs(0.5 * q32.astype(np.float64) - 0.5 * q) / bound)
    r = np.concatenate(ratios)
    assert r.max() < 0.7, float(r.max())
    assert np.median(r) > 1e-3, float(np.median(r))

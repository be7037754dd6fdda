"""Pins of the CPU reference against facts it does not compute itself.

Each test checks the oracle against mathematics fixed independently of its code:
closed-form images, compositing identities, quadrature, a third-party rotation routine,
numerical derivatives, and the paper's exactness claim for the local kernel (Sec. 3.3
"Local Optimization Kernel": the changed Gaussians get the same gradients as in a
full-scene step).  They run on the CPU only.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import scenes
from scenes import Camera, Scene

Y00 = 0.5 / math.sqrt(math.pi)


def make_scene(means, log_scales, quats, opacity, dc, sh_degree=0, rest=None):
    n = len(means)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((K, 3, n), np.float32)
    sh[0] = np.asarray(dc, np.float32).T
    if rest is not None:
        sh[1:] = rest
    logit = np.log(np.asarray(opacity, np.float64) / (1 - np.asarray(opacity, np.float64)))
    return Scene(np.asarray(means, np.float32).T, np.asarray(log_scales, np.float32).T,
                 np.asarray(quats, np.float32).T, logit.astype(np.float32), sh, sh_degree)


def dc_for_rgb(rgb):
    return (np.asarray(rgb, np.float64) - 0.5) / Y00


def rot_camera(W=64, H=48, f=60.0, angles=(0.3, -0.2, 0.1), center=(0.2, -0.1, -4.0)):
    R = Rotation.from_euler("xyz", angles).as_matrix().astype(np.float32)
    c = np.asarray(center, np.float64)
    t = (-(R.astype(np.float64) @ c)).astype(np.float32)
    return Camera(R, t, f, f * 1.1, W / 2 + 0.25, H / 2 - 0.5, W, H)


def closed_form_isotropic(mu, s, o, rgb, cam, bg):
    """Pixel image of one isotropic Gaussian: Sigma2 = s^2 J J^T + 0.3 I, where J is
    the perspective Jacobian at the centre (no rotation enters for an isotropic
    Gaussian because R R^T = I)."""
    R = cam.R.astype(np.float64)
    p = R @ np.asarray(mu, np.float64) + cam.t.astype(np.float64)
    X, Y, Z = p
    u = cam.fx * X / Z + cam.cx
    v = cam.fy * Y / Z + cam.cy
    JJt = np.array([[cam.fx ** 2 * (1 / Z ** 2 + X ** 2 / Z ** 4), cam.fx * cam.fy * X * Y / Z ** 4],
                    [cam.fx * cam.fy * X * Y / Z ** 4, cam.fy ** 2 * (1 / Z ** 2 + Y ** 2 / Z ** 4)]])
    S2 = s * s * JJt + 0.3 * np.eye(2)
    Si = np.linalg.inv(S2)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    dx = xs + 0.5 - u
    dy = ys + 0.5 - v
    q = Si[0, 0] * dx * dx + 2 * Si[0, 1] * dx * dy + Si[1, 1] * dy * dy
    a = np.minimum(0.99, o * np.exp(-0.5 * q))
    a = np.where(a >= 1 / 255, a, 0.0)
    img = np.asarray(rgb)[:, None, None] * a + (1 - a) * np.asarray(bg)[:, None, None]
    return img, S2, (u, v)


def perm_camera(W=64, H=48, f=60.0):
    """A camera whose float32 rotation is exactly orthonormal (a signed permutation),
    placed off the origin and looking along world -x."""
    R = np.array([[0, 1, 0], [0, 0, -1], [-1, 0, 0]], np.float32)
    c = np.array([4.0, 0.125, -0.25])
    t = (-(R.astype(np.float64) @ c)).astype(np.float32)
    return Camera(R, t, f, f * 1.1, W / 2 + 0.25, H / 2 - 0.5, W, H)


# ------------------------------------------------------------------ A: one isotropic Gaussian
@pytest.mark.parametrize("mu", [(0.0, 0.0, 0.0), (0.35, -0.2, 0.5), (-0.6, 0.45, -0.3)])
@pytest.mark.parametrize("camera,tol", [(perm_camera, 1e-12), (rot_camera, 2e-6)])
def test_single_isotropic_closed_form(orc, mu, camera, tol):
    """The closed form needs R R^T = I; the general float32 rotation is orthonormal only
    to float32 precision, hence its looser tolerance."""
    cam = camera()
    s, o, rgb, bg = 0.08, 0.8, (0.9, 0.3, 0.6), (0.1, 0.2, 0.3)
    q = Rotation.random(random_state=3).as_quat()  # any rotation: isotropic
    sc = make_scene([mu], [[math.log(s)] * 3], [[q[3], q[0], q[1], q[2]]], [o], [dc_for_rgb(rgb)])
    # the float32 inputs are what both sides see
    s32 = float(np.exp(np.float64(sc.log_scales[0, 0])))
    o32 = 1 / (1 + math.exp(-float(sc.opacity_logit[0])))
    rgb32 = Y00 * sc.sh[0, :, 0].astype(np.float64) + 0.5
    expect, S2, (u, v) = closed_form_isotropic(sc.means[:, 0], s32, o32, rgb32, cam, bg)
    r = orc.render(sc, cam, bg)
    np.testing.assert_allclose(r["image"], expect, rtol=0, atol=tol)
    assert (r["image"] != np.asarray(bg)[:, None, None]).any()
    pp = orc.preprocess(sc, cam)
    np.testing.assert_allclose([pp["cov_a"][0], pp["cov_b"][0], pp["cov_c"][0]], [S2[0, 0], S2[0, 1], S2[1, 1]],
                               rtol=tol)
    np.testing.assert_allclose([pp["u"][0], pp["v"][0]], [u, v], rtol=1e-13)
    # conic is the inverse of the screen covariance
    Si = np.array([[pp["A"][0], pp["B"][0]], [pp["B"][0], pp["C"][0]]])
    S2o = np.array([[pp["cov_a"][0], pp["cov_b"][0]], [pp["cov_b"][0], pp["cov_c"][0]]])
    np.testing.assert_allclose(Si @ S2o, np.eye(2), atol=1e-12)


def test_anisotropic_on_axis_closed_form(orc):
    """On the optical axis J = diag(fx/Z, fy/Z) (third column zero), so Sigma2 is the
    upper 2x2 block of R diag(s^2) R^T scaled by f^2/Z^2, plus 0.3.  A rotation by theta
    about z mixes s1 and s2 by cos/sin; one about x mixes s2 and s3."""
    cam = Camera(np.eye(3), (0, 0, 4), 100, 120, 32, 32, 64, 64)
    s = np.array([0.05, 0.12, 0.2])
    th = 0.7
    qz = (math.cos(th / 2), 0, 0, math.sin(th / 2))
    qx = (math.cos(th / 2), math.sin(th / 2), 0, 0)
    sc = make_scene([(0, 0, 0), (0, 0, 0.5)], [np.log(s)] * 2, [qz, qx], [0.5, 0.5], [dc_for_rgb((0.5,) * 3)] * 2)
    s32 = np.exp(sc.log_scales[:, 0].astype(np.float64))
    pp = orc.preprocess(sc, cam)
    c, sn = math.cos(th), math.sin(th)
    # recompute the quaternion angle from the float32 inputs
    qz32 = sc.quats[:, 0].astype(np.float64)
    qz32 /= np.linalg.norm(qz32)
    thz = 2 * math.atan2(qz32[3], qz32[0])
    c, sn = math.cos(thz), math.sin(thz)
    Z = 4.0
    blk = np.array([[c * c * s32[0] ** 2 + sn * sn * s32[1] ** 2, c * sn * (s32[0] ** 2 - s32[1] ** 2)],
                    [c * sn * (s32[0] ** 2 - s32[1] ** 2), sn * sn * s32[0] ** 2 + c * c * s32[1] ** 2]])
    F = np.diag([cam.fx / Z, cam.fy / Z])
    S2 = F @ blk @ F + 0.3 * np.eye(2)
    np.testing.assert_allclose([pp["cov_a"][0], pp["cov_b"][0], pp["cov_c"][0]], [S2[0, 0], S2[0, 1], S2[1, 1]],
                               rtol=1e-12)
    qx32 = sc.quats[:, 1].astype(np.float64)
    qx32 /= np.linalg.norm(qx32)
    thx = 2 * math.atan2(qx32[1], qx32[0])
    c, sn = math.cos(thx), math.sin(thx)
    Z = 4.5
    blk = np.array([[s32[0] ** 2, 0.0], [0.0, c * c * s32[1] ** 2 + sn * sn * s32[2] ** 2]])
    F = np.diag([cam.fx / Z, cam.fy / Z])
    S2 = F @ blk @ F + 0.3 * np.eye(2)
    np.testing.assert_allclose([pp["cov_a"][1], pp["cov_b"][1], pp["cov_c"][1]], [S2[0, 0], S2[0, 1], S2[1, 1]],
                               rtol=1e-12, atol=1e-12)


def test_covariance_against_numeric_jacobian_and_scipy_rotation(orc):
    """Sigma2 = J Rcam Sigma Rcam^T J^T + 0.3 I with J the derivative of the pinhole map
    taken by central differences and Sigma built with scipy's quaternion rotation."""
    rng = np.random.default_rng(7)
    cam = rot_camera(W=96, H=80, f=90.0)
    n = 40
    sc = make_scene(rng.uniform(-0.5, 0.5, (n, 3)), rng.normal(-2.5, 0.4, (n, 3)), rng.normal(size=(n, 4)),
                    rng.uniform(0.2, 0.9, n), rng.normal(size=(n, 3)))
    pp = orc.preprocess(sc, cam)
    R = cam.R.astype(np.float64)
    t = cam.t.astype(np.float64)

    def proj(x):
        pc = R @ x + t
        return np.array([cam.fx * pc[0] / pc[2] + cam.cx, cam.fy * pc[1] / pc[2] + cam.cy])

    checked = 0
    for i in range(n):
        if not pp["visible"][i] or pp["flags"][i] & (orc.F_CLAMPX | orc.F_CLAMPY):
            continue
        mu = sc.means[:, i].astype(np.float64)
        h = 1e-5
        Jw = np.stack([(proj(mu + h * e) - proj(mu - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        q = sc.quats[:, i].astype(np.float64)
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        s = np.exp(sc.log_scales[:, i].astype(np.float64))
        Sig = Rq @ np.diag(s * s) @ Rq.T
        S2 = Jw @ Sig @ Jw.T + 0.3 * np.eye(2)
        got = np.array([[pp["cov_a"][i], pp["cov_b"][i]], [pp["cov_b"][i], pp["cov_c"][i]]])
        np.testing.assert_allclose(got, S2, rtol=1e-7, atol=1e-7)
        np.testing.assert_allclose([pp["u"][i], pp["v"][i]], proj(mu), rtol=1e-12)
        checked += 1
    assert checked > 20


def test_clamped_jacobian_covariance_closed_form(orc):
    """Past the lateral limit the Jacobian uses the clamped ratio: X~/Z = sign(X) 1.3 (W/2)/fx
    (and Y~/Z likewise with H and fy), while the projected centre keeps the true ratio.
    For an isotropic Gaussian under an identity camera rotation, Sigma2 = s^2 J J^T + 0.3 I
    with J = [[fx/Z, 0, -fx X~/Z^2], [0, fy/Z, -fy Y~/Z^2]], written out here by hand."""
    W, H, fx, fy = 64, 40, 50.0, 45.0
    cam = Camera(np.eye(3), (0, 0, 4), fx, fy, W / 2, H / 2, W, H)
    lx, ly = 1.3 * (W / 2) / fx, 1.3 * (H / 2) / fy      # 0.832 and 0.5777...
    # centres (camera space: Z = 4 + z): clamped in x (both signs), in y (both signs),
    # in both, and one inside both limits
    mus = [(4.2, 0.3, 0.5), (-4.0, -0.2, 0.0), (0.4, 3.1, 0.2), (-0.3, -3.6, 1.0), (5.0, 3.8, 0.3), (0.5, 0.4, 0.0)]
    s = 0.3
    q = (1.0, 0.0, 0.0, 0.0)
    sc = make_scene(mus, [[math.log(s)] * 3] * len(mus), [q] * len(mus), [0.7] * len(mus),
                    [dc_for_rgb((0.5,) * 3)] * len(mus))
    pp = orc.preprocess(sc, cam)
    want_flags = [(1, 0), (1, 0), (0, 1), (0, 1), (1, 1), (0, 0)]
    for i, (cx_, cy_) in enumerate(want_flags):
        assert bool(pp["flags"][i] & orc.F_CLAMPX) == bool(cx_), i
        assert bool(pp["flags"][i] & orc.F_CLAMPY) == bool(cy_), i
        mu = sc.means[:, i].astype(np.float64)
        s32 = float(np.exp(np.float64(sc.log_scales[0, i])))
        X, Y, Z = mu[0], mu[1], mu[2] + 4.0
        rx = X / Z if not cx_ else math.copysign(lx, X)
        ry = Y / Z if not cy_ else math.copysign(ly, Y)
        a = s32 ** 2 * (fx / Z) ** 2 * (1 + rx * rx) + 0.3
        b = s32 ** 2 * (fx / Z) * (fy / Z) * rx * ry
        c = s32 ** 2 * (fy / Z) ** 2 * (1 + ry * ry) + 0.3
        np.testing.assert_allclose([pp["cov_a"][i], pp["cov_b"][i], pp["cov_c"][i]], [a, b, c], rtol=1e-12,
                                   atol=1e-14)
        np.testing.assert_allclose([pp["u"][i], pp["v"][i]], [fx * X / Z + W / 2, fy * Y / Z + H / 2], rtol=1e-13)


# ------------------------------------------------------------------ B, C: compositing
def test_two_gaussians_composite(orc):
    cam = Camera(np.eye(3), (0, 0, 4), 64, 64, 32, 32, 64, 64)
    rgb1, rgb2, bg = (0.9, 0.1, 0.2), (0.2, 0.7, 0.4), (0.3, 0.3, 0.5)
    sc = make_scene([(0.0, 0.0, 0.0), (0.05, 0.02, 0.6)], [[math.log(0.1)] * 3, [math.log(0.15)] * 3],
                    [(1, 0, 0, 0), (1, 0, 0, 0)], [0.6, 0.7], [dc_for_rgb(rgb1), dc_for_rgb(rgb2)])
    r = orc.render(sc, cam, bg)
    # closed forms of each alone with bg = 0 give their alpha * rgb maps
    a = []
    for i in range(2):
        s = float(np.exp(np.float64(sc.log_scales[0, i])))
        o = 1 / (1 + math.exp(-float(sc.opacity_logit[i])))
        one, _, _ = closed_form_isotropic(sc.means[:, i], s, o, (1.0, 1.0, 1.0), cam, (0.0, 0.0, 0.0))
        a.append(one[0])
    c1 = Y00 * sc.sh[0, :, 0].astype(np.float64) + 0.5
    c2 = Y00 * sc.sh[0, :, 1].astype(np.float64) + 0.5
    expect = (c1[:, None, None] * a[0] + c2[:, None, None] * a[1] * (1 - a[0])
              + np.asarray(bg)[:, None, None] * (1 - a[0]) * (1 - a[1]))
    np.testing.assert_allclose(r["image"], expect, atol=1e-12)
    # the nearer Gaussian is first whatever the index order
    r2 = orc.render(sc.take([1, 0]), cam, bg)
    np.testing.assert_allclose(r2["image"], r["image"], atol=1e-15)


def stop_stack_scene():
    """Three Gaussians centred exactly on the pixel centre (31.5 + 0.5 = 32 -> use a
    -0.5 px shift) at depths 3, 4, 5: alphas 0.99 (clamped), 0.98, 0.9.  T goes 1 ->
    0.01 -> 2e-4, and the third would take it to 2e-5 < 1e-4, so it is not blended."""
    fx = 64.0
    cam = Camera(np.eye(3), (0, 0, 0), fx, fx, 32, 32, 64, 64)
    means, ls = [], []
    for Z in (3.0, 4.0, 5.0):
        means.append((-0.5 * Z / fx, -0.5 * Z / fx, Z))
        ls.append([math.log(0.2)] * 3)
    ops = [0.9999, 0.98, 0.9]
    cols = [(0.8, 0.1, 0.1), (0.1, 0.8, 0.1), (0.1, 0.1, 0.8)]
    sc = make_scene(means, ls, [(1, 0, 0, 0)] * 3, ops, [dc_for_rgb(c) for c in cols])
    return sc, cam


def test_stop_rule_stack(orc):
    sc, cam = stop_stack_scene()
    bg = (0.25, 0.5, 0.75)
    pix = np.array([[31, 31]], np.int32)
    dl = np.array([[1.0, -2.0, 0.5]])
    r = orc.render(sc, cam, bg, pixels=pix, dL_dC=dl)
    o2 = 1 / (1 + math.exp(-float(sc.opacity_logit[1])))
    c = [Y00 * sc.sh[0, :, i].astype(np.float64) + 0.5 for i in range(3)]
    T1 = 1 - 0.99
    T2 = T1 * (1 - o2)
    expect = 0.99 * c[0] + T1 * o2 * c[1] + T2 * np.asarray(bg)
    assert r["ncontrib"][0] == 2
    np.testing.assert_allclose(r["T"][0], T2, rtol=1e-12)
    np.testing.assert_allclose(r["rgb"][0], expect, atol=1e-12)
    assert r["T"][0] >= 1e-4
    # the third Gaussian is not blended: it gets no gradient at all
    assert np.all(r["grad2d"][2] == 0)
    # the first is clamped: zero opacity gradient, colour gradient 0.99 * dL/dC
    assert r["grad2d"][0, 5] == 0
    np.testing.assert_allclose(r["grad2d"][0, 6:9], 0.99 * dl[0], rtol=1e-12)
    np.testing.assert_allclose(r["grad2d"][1, 6:9], T1 * o2 * dl[0], rtol=1e-12)
    # dC/dalpha_2 = T_2 c_2 - T_final bg/(1 - alpha_2), alpha_2 = o2 at the centre
    dCda = T1 * c[1] - T2 * np.asarray(bg) / (1 - o2)
    np.testing.assert_allclose(r["grad2d"][1, 5], float(dl[0] @ dCda), rtol=1e-10)


# ------------------------------------------------------------------ D: spherical harmonics
def test_sh_orthonormal_by_quadrature(orc):
    xg, wg = np.polynomial.legendre.leggauss(12)       # exact for degree <= 23 in cos(theta)
    nphi = 24
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct = np.repeat(xg, nphi)
    w = np.repeat(wg, nphi) * (2 * np.pi / nphi)
    st = np.sqrt(1 - ct * ct)
    ph = np.tile(phi, len(xg))
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=1)
    Y = orc.sh_basis(d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_degree0_colour_closed_form(orc):
    w = scenes.tiny(n=200)
    pp = orc.preprocess(w.scene, w.cameras[0])
    rgb = np.maximum(0.0, Y00 * w.scene.sh[0].astype(np.float64) + 0.5)
    vis = pp["visible"]
    np.testing.assert_allclose(np.stack([pp["r"], pp["g"], pp["b"]])[:, vis], rgb[:, vis], rtol=1e-14)


def test_sh_band1_direction(orc):
    """A degree-1 coefficient on Y_{1,0} (the z polynomial) adds C1 * dir_z to the
    colour, with dir the unit vector from the camera centre to the mean."""
    cam = rot_camera()
    mu = (0.3, -0.2, 0.4)
    rest = np.zeros((3, 3, 1), np.float32)
    rest[1, :, 0] = (0.4, -0.3, 0.2)             # k = 2 -> (l=1, m=0)
    sc = make_scene([mu], [[math.log(0.05)] * 3], [(1, 0, 0, 0)], [0.5], [dc_for_rgb((0.5, 0.5, 0.5))], 1, rest)
    pp = orc.preprocess(sc, cam)
    campos = -cam.R.astype(np.float64).T @ cam.t.astype(np.float64)
    d = sc.means[:, 0].astype(np.float64) - campos
    d /= np.linalg.norm(d)
    C1 = math.sqrt(3 / (4 * math.pi))
    expect = Y00 * sc.sh[0, :, 0].astype(np.float64) + 0.5 + C1 * d[2] * sc.sh[2, :, 0].astype(np.float64)
    np.testing.assert_allclose([pp["r"][0], pp["g"][0], pp["b"][0]], expect, rtol=1e-13)


# ------------------------------------------------------------------ F: invariants
def test_invariants_weights_and_background(orc):
    w = scenes.tiny(n=400, width=48, height=40)
    sc = w.scene.copy()
    sc.sh[0] = dc_for_rgb(np.ones((3, sc.n)))      # every colour = 1
    cam = w.cameras[0]
    r0 = orc.render(sc, cam, (0, 0, 0))
    r1 = orc.render(sc, cam, (1, 1, 1))
    # sum of weights + T_final = 1 (I1): white scene on black = 1 - T
    np.testing.assert_allclose(r0["image"], np.broadcast_to(1 - r0["T_image"], r0["image"].shape), atol=1e-12)
    # background enters with weight T_final
    np.testing.assert_allclose(r1["image"] - r0["image"], np.broadcast_to(r0["T_image"], r0["image"].shape),
                               atol=1e-12)
    assert np.all(r0["T"] >= 1e-4) and np.all(r0["T"] <= 1)          # I2
    # I4: pixels of the coloured scene lie in the hull of [0, 1] colours and bg
    rc = orc.render(w.scene, cam, (0.2, 0.4, 0.6))
    assert rc["image"].min() >= 0 and rc["image"].max() <= 1 + 1e-12


def test_invariant_shuffle(orc):
    w = scenes.tiny(n=300, width=40, height=32)
    cam = w.cameras[0]
    r = orc.render(w.scene, cam)
    perm = np.random.default_rng(1).permutation(w.scene.n)
    pp = orc.preprocess(w.scene, cam)
    z = pp["z32"][pp["visible"]]
    assert len(np.unique(z)) == len(z), "tie-free scene expected"
    r2 = orc.render(w.scene.take(perm), cam)
    np.testing.assert_array_equal(r["image"], r2["image"])


def test_invariant_empty_near_and_transparent(orc):
    cam = Camera(np.eye(3), (0, 0, 4), 32, 32, 16, 16, 32, 32)
    bg = (0.3, 0.6, 0.9)
    empty = make_scene(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)), np.zeros(0), np.zeros((0, 3)))
    r = orc.render(empty, cam, bg)
    np.testing.assert_array_equal(r["image"], np.broadcast_to(np.asarray(bg)[:, None, None], (3, 32, 32)))
    # a Gaussian behind the near plane (z = 0.1 in camera space) and one with
    # opacity below 1/255 contribute nothing
    sc = make_scene([(0, 0, -3.9), (0, 0, 0)], [[math.log(0.3)] * 3] * 2, [(1, 0, 0, 0)] * 2,
                    [0.9, 0.0035], [dc_for_rgb((1, 0, 0))] * 2)
    r = orc.render(sc, cam, bg)
    np.testing.assert_array_equal(r["image"], np.broadcast_to(np.asarray(bg)[:, None, None], (3, 32, 32)))
    pp = orc.preprocess(sc, cam)
    assert not pp["visible"].any()


def test_invariant_joint_translation(orc):
    w = scenes.tiny(n=300, width=40, height=32)
    cam = w.cameras[0]
    d = np.array([0.5, -0.25, 1.0])
    params = [np.asarray(a, np.float64).copy() for a in w.scene.param_arrays()]
    shifted = [a.copy() for a in params]
    shifted[0] = shifted[0] + d[:, None]
    cam2 = Camera(cam.R, cam.t.astype(np.float64) - cam.R.astype(np.float64) @ d, cam.fx, cam.fy, cam.cx, cam.cy,
                  cam.width, cam.height)
    assert np.allclose(cam2.t.astype(np.float64), cam.t.astype(np.float64) - cam.R.astype(np.float64) @ d, atol=0)
    r = orc.render(w.scene, cam, params=tuple(params))
    r2 = orc.render(w.scene, cam2, params=tuple(shifted))
    np.testing.assert_allclose(r2["image"], r["image"], atol=1e-9)


# ------------------------------------------------------------------ G: finite differences
def _fd_check(orc, sc, cams, bg, dls, rng, n_per_group=10, rel=1e-6, pick=None):
    """Central differences in double, h = 5e-6 max(1, |theta|); a sample counts only if
    every pixel's contributor count and near-threshold flag agree at theta +- h."""
    g = orc.gradients(sc, cams, dls, bg)
    base = [np.asarray(a, np.float64).copy() for a in sc.param_arrays()]
    names = ["means", "log_scales", "quats", "opacity_logit", "sh"]

    def render_all(params):
        imgs, dec = [], []
        for cam in cams:
            r = orc.render(sc, cam, bg, params=tuple(params))
            imgs.append(r["image"])
            dec.append(r["ncontrib"])
            dec.append(r["flag"])
        return imgs, np.concatenate(dec)

    # Gaussians that blend somewhere
    contributes = np.zeros(sc.n, bool)
    for cam, dl in zip(cams, dls):
        r = orc.render(sc, cam, bg, dL_dC=dl)
        contributes |= np.abs(r["grad2d"]).sum(1) > 0
    cand = np.nonzero(contributes)[0] if pick is None else pick
    checked = skipped = 0
    for gi, name in enumerate(names):
        arr = base[gi]
        ncomp = arr.reshape(-1, sc.n).shape[0]
        for _ in range(n_per_group):
            i = int(rng.choice(cand))
            c = int(rng.integers(ncomp))
            val = arr.reshape(ncomp, sc.n)[c, i]
            h = 5e-6 * max(1.0, abs(val))
            pp_ = [a.copy() for a in base]
            pm_ = [a.copy() for a in base]
            pp_[gi].reshape(ncomp, sc.n)[c, i] += h
            pm_[gi].reshape(ncomp, sc.n)[c, i] -= h
            ip, dp = render_all(pp_)
            im, dm = render_all(pm_)
            if not np.array_equal(dp, dm):     # a decision changed inside [theta-h, theta+h]
                skipped += 1
                continue
            # difference the images first: the loss itself is a large sum
            fd = sum(float(((a - b) * dl).sum()) for a, b, dl in zip(ip, im, dls)) / (2 * h)
            an = g[name].reshape(ncomp, sc.n)[c, i]
            tol = rel * max(abs(fd), abs(an)) + 1e-10
            assert abs(an - fd) <= tol, (name, c, i, an, fd)
            checked += 1
    assert checked >= 4 * n_per_group, (checked, skipped)


def test_fd_gradients_degree0(orc):
    rng = np.random.default_rng(11)
    w = scenes.tiny(n=80, width=32, height=32)
    dl = [rng.normal(size=(3, 32, 32))]
    _fd_check(orc, w.scene, w.cameras, (0.0, 0.0, 0.0), dl, rng)


def test_fd_gradients_degree3_two_views_background(orc):
    rng = np.random.default_rng(12)
    w = scenes.fd_scene(n=70, res=28)
    cams = [w.cameras[0], rot_camera(W=28, H=24, f=30.0)]
    dl = [rng.normal(size=(3, c.height, c.width)) for c in cams]
    _fd_check(orc, w.scene, cams, (0.2, 0.5, 0.3), dl, rng)


def test_fd_gradients_jacobian_clamp_and_sh_clamp(orc):
    """Gaussians far off to the side (lateral ratio clamped) but large enough to reach
    the image, and SH coefficients that push some channels below zero."""
    rng = np.random.default_rng(13)
    cam = Camera(np.eye(3), (0, 0, 4), 40, 40, 16, 16, 32, 32)
    n = 30
    means = np.stack([rng.uniform(-4.5, 4.5, n), rng.uniform(-0.5, 0.5, n), rng.uniform(-1, 1, n)], 1)
    ls = rng.normal(-0.7, 0.3, (n, 3))
    rest = rng.normal(0, 0.8, (3, 3, n)).astype(np.float32)
    sc = make_scene(means, ls, rng.normal(size=(n, 4)), rng.uniform(0.3, 0.95, n), rng.normal(0, 1.2, (n, 3)), 1, rest)
    pp = orc.preprocess(sc, cam)
    clampx = (pp["flags"] & orc.F_CLAMPX) != 0
    shc = (pp["flags"] & (orc.F_SHCLAMP_R | orc.F_SHCLAMP_G | orc.F_SHCLAMP_B)) != 0
    dl = [rng.normal(size=(3, 32, 32))]
    r = orc.render(sc, cam, dL_dC=dl[0])
    contrib = np.abs(r["grad2d"]).sum(1) > 0
    assert (clampx & contrib).sum() >= 2 and (shc & contrib).sum() >= 2
    pick = np.nonzero(contrib & (clampx | shc))[0]
    _fd_check(orc, sc, [cam], (0.0, 0.0, 0.0), dl, rng, pick=pick)


def test_fd_gradients_y_clamped(orc):
    """Gaussians far above and below the view (vertical ratio clamped, so Y~ = Z Y~/Z
    depends on the depth only) that still reach the image; every means component of
    each such Gaussian is checked against central differences."""
    rng = np.random.default_rng(17)
    cam = Camera(np.eye(3), (0, 0, 4), 40, 40, 16, 12, 32, 24)
    n = 40
    means = np.stack([rng.uniform(-0.6, 0.6, n), rng.choice([-1.0, 1.0], n) * rng.uniform(2.2, 4.0, n),
                      rng.uniform(-1, 1, n)], 1)
    ls = rng.normal(-0.6, 0.25, (n, 3))
    sc = make_scene(means, ls, rng.normal(size=(n, 4)), rng.uniform(0.4, 0.95, n), rng.uniform(-1, 1, (n, 3)))
    pp = orc.preprocess(sc, cam)
    clampy = (pp["flags"] & orc.F_CLAMPY) != 0
    dl = rng.normal(size=(3, 24, 32))
    r = orc.render(sc, cam, dL_dC=dl)
    contrib = np.abs(r["grad2d"]).sum(1) > 0
    pick = np.nonzero(contrib & clampy)[0]
    assert len(pick) >= 4, len(pick)
    g = orc.gradients(sc, [cam], [dl])
    base = [np.asarray(a, np.float64).copy() for a in sc.param_arrays()]
    checked = 0
    for i in pick:
        for c in range(3):
            val = base[0][c, i]
            h = 5e-6 * max(1.0, abs(val))
            pp_, pm_ = [a.copy() for a in base], [a.copy() for a in base]
            pp_[0][c, i] += h
            pm_[0][c, i] -= h
            rp = orc.render(sc, cam, params=tuple(pp_))
            rm = orc.render(sc, cam, params=tuple(pm_))
            if not (np.array_equal(rp["ncontrib"], rm["ncontrib"]) and np.array_equal(rp["flag"], rm["flag"])):
                continue
            fd = float(((rp["image"] - rm["image"]) * dl).sum()) / (2 * h)
            an = g["means"][c, i]
            assert abs(an - fd) <= 1e-6 * max(abs(fd), abs(an)) + 1e-10, (c, i, an, fd)
            checked += 1
    assert checked >= 3 * len(pick) - 2, checked


# ------------------------------------------------------------------ K: the local-kernel claim
def test_local_gradients_equal_full_on_changed_set(orc):
    """Gradients of the changed Gaussians from the pixels of their tile mask only equal
    their full-image gradients (Sec. 3.3): every pixel where a Gaussian can reach
    alpha >= 1/255 lies inside its tile rectangle."""
    rng = np.random.default_rng(5)
    w = scenes.tiny(n=600, width=96, height=80)
    sc, cam = w.scene, w.cameras[0]
    a0 = 520
    pp = orc.preprocess(sc, cam)
    f32 = lambda k: pp[k].astype(np.float32)
    b = orc.bin_reference(f32("u"), f32("v"), f32("rx"), f32("ry"), pp["z32"], pp["visible"], cam.width,
                          cam.height, active=(a0, sc.n), use_mask=True)
    TX, TY = orc.tile_grid(cam.width, cam.height)
    tmask = b["mask"].reshape(TY, TX)
    pmask = np.kron(tmask, np.ones((16, 16), bool))[:cam.height, :cam.width]
    assert 0.05 < pmask.mean() < 0.95
    tgt = w.targets[0][:, :cam.height, :cam.width] if w.targets[0].shape[1:] == (cam.height, cam.width) else \
        rng.uniform(size=(3, cam.height, cam.width))
    img = orc.render(sc, cam)["image"]
    _, dl_full = orc.l1_loss_grad(img, tgt)
    _, dl_loc = orc.l1_loss_grad(img, tgt, pixel_mask=pmask)
    gf = orc.gradients(sc, [cam], [dl_full])
    gl = orc.gradients(sc, [cam], [dl_loc])
    for k in ("means", "log_scales", "quats", "opacity_logit", "sh"):
        act_f = gf[k][..., a0:]
        act_l = gl[k][..., a0:]
        np.testing.assert_allclose(act_l, act_f, rtol=1e-12, atol=1e-14)
    assert np.abs(gf["means"][..., a0:]).max() > 0


# ------------------------------------------------------------------ H: binning reference
def test_bin_reference_covers_every_blend(orc):
    """Every (pixel, Gaussian) pair the brute-force renderer blends appears in that
    pixel's tile list, ranges partition [0, P), and lists are depth ordered."""
    w = scenes.tiny(n=300, width=72, height=56)
    sc, cam = w.scene, w.cameras[0]
    pp = orc.preprocess(sc, cam)
    f32 = lambda k: pp[k].astype(np.float32)
    b = orc.bin_reference(f32("u"), f32("v"), f32("rx"), f32("ry"), pp["z32"], pp["visible"], cam.width,
                          cam.height)
    TX, TY = orc.tile_grid(cam.width, cam.height)
    x0, x1, y0, y1 = b["rects"]
    assert b["n_pairs"] == int(((x1 - x0) * (y1 - y0))[pp["visible"]].sum())
    rg = b["ranges"]
    nonempty = rg[:, 1] > rg[:, 0]
    assert rg[nonempty, 1].max() == b["n_pairs"]
    order = np.argsort(rg[nonempty, 0])
    st, en = rg[nonempty, 0][order], rg[nonempty, 1][order]
    assert st[0] == 0 and np.all(st[1:] == en[:-1])
    for t in np.nonzero(nonempty)[0]:
        ids = b["values"][rg[t, 0]:rg[t, 1]]
        z = pp["z32"][ids]
        assert np.all((z[1:] > z[:-1]) | ((z[1:] == z[:-1]) & (ids[1:] > ids[:-1])))
    # blends found by the renderer, one Gaussian at a time
    for i in np.nonzero(pp["visible"])[0][:60]:
        r = orc.render(sc.take([i]), cam)
        hit = r["ncontrib"].reshape(cam.height, cam.width) > 0
        ys, xs = np.nonzero(hit)
        tiles = np.unique((ys // 16) * TX + xs // 16)
        for t in tiles:
            assert i in b["values"][rg[t, 0]:rg[t, 1]]


# ------------------------------------------------------------------ I: Adam, loss
def test_adam_first_and_second_step_closed_form(orc):
    rng = np.random.default_rng(3)
    n = 10
    p = {"a": rng.normal(size=(3, n)), "b": rng.normal(size=n)}
    g = {"a": rng.normal(size=(3, n)), "b": rng.normal(size=n)}
    z = {k: np.zeros_like(v) for k, v in p.items()}
    lrs = {"a": 1e-3, "b": 5e-2}
    rows = np.arange(4, n)
    P1, M1, V1 = orc.adam_step(p, g, z, z, 1, lrs, rows=rows)
    for k in p:
        d = P1[k][..., rows] - p[k][..., rows]
        np.testing.assert_allclose(d, -lrs[k] * g[k][..., rows] / (np.abs(g[k][..., rows]) + 1e-15), rtol=1e-12)
        np.testing.assert_array_equal(P1[k][..., :4], p[k][..., :4])
        np.testing.assert_array_equal(M1[k][..., :4], 0)
    # second step with the same gradient: m = g(1 - b1^2), v = g^2(1 - b2^2) -> mhat = g,
    # vhat = g^2 again, so the step is the same size
    P2, _, _ = orc.adam_step(P1, g, M1, V1, 2, lrs, rows=rows)
    for k in p:
        d = P2[k][..., rows] - P1[k][..., rows]
        np.testing.assert_allclose(d, -lrs[k] * g[k][..., rows] / (np.abs(g[k][..., rows]) + 1e-15), rtol=1e-9)


def test_l1_loss_grad(orc):
    img = np.zeros((3, 2, 2))
    tgt = np.array([[[0.5, 0.0], [-1, 0]]] * 3)
    loss, g = orc.l1_loss_grad(img, tgt)
    assert loss == pytest.approx(3 * 1.5 / 12)
    np.testing.assert_array_equal(g[0], np.array([[-1, 0], [1, 0]]) / 12)

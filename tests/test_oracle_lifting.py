"""Pins of the change-lifting steps in the CPU reference: mask dilation (Supp.
"Detecting Changes in 2D": dilate by 2% of the width with a kernel of ones, threshold
at 0) against brute force and closed forms, and the majority vote (Supp. "Identifying
Changed 3D Regions via Majority Voting": g_i changed iff 4/3 o_i < |I| < 2 c_i) on
hand-built cameras and masks."""
import numpy as np

import oracle
import scenes


def _dilate_brute(m, r):
    V, H, W = m.shape
    out = np.zeros_like(m, dtype=np.uint8)
    for v in range(V):
        for y in range(H):
            for x in range(W):
                acc = 0
                for dy in range(-r, r + 1):
                    for dx in range(-r, r + 1):
                        yy, xx = y + dy, x + dx
                        if 0 <= yy < H and 0 <= xx < W:
                            acc += int(m[v, yy, xx] != 0)
                out[v, y, x] = 1 if acc > 0 else 0
    return out


def test_dilation_equals_brute_force():
    rng = np.random.default_rng(0)
    for (V, H, W), r, p in (((2, 13, 20), 3, 0.02), ((1, 9, 31), 5, 0.01), ((1, 17, 17), 1, 0.1), ((1, 7, 8), 9, 0.05)):
        m = (rng.random((V, H, W)) < p).astype(np.uint8)
        np.testing.assert_array_equal(oracle.dilate_masks(m, r), _dilate_brute(m, r))


def test_dilation_closed_forms():
    m = np.zeros((1, 30, 40), np.uint8)
    m[0, 2, 37] = 1
    d = oracle.dilate_masks(m, 4)
    want = np.zeros_like(m)
    want[0, 0:7, 33:40] = 1                     # the 9 x 9 square, cut at the borders
    np.testing.assert_array_equal(d, want)
    assert not oracle.dilate_masks(np.zeros((2, 5, 6), np.uint8), 3).any()
    m = (np.random.default_rng(1).random((1, 11, 13)) < 0.3).astype(np.uint8)
    np.testing.assert_array_equal(oracle.dilate_masks(m, 0), m)
    assert [oracle.dilation_radius(w) for w in (640, 1250, 1280, 1920)] == [13, 25, 26, 38]


def test_majority_vote_counts_and_thresholds():
    """Four cameras on a ring of radius 4 looking at the origin, 64 x 48, f = 64."""
    cams = scenes.ring_cameras(4, 4.0, width=64, height=48, fx=64.0)
    pts = np.array([[0.0, 0.0, 0.0],        # every view, at the centre pixel (32, 24)
                    [0.0, 0.0, -3.9],       # 0.1 in front of camera 0 (near plane: outside),
                                            # at the centre of camera 2 (depth 7.9), and
                                            # u = 32 -+ 64 * 3.9 / 4 off the image of 1 and 3
                    [0.0, 2.9, 0.0]]).T     # v = 24 + 64 * 2.9 / 4 = 70.4 > 48: outside all
    masks = np.zeros((4, 48, 64), np.uint8)
    masks[:, 24, 32] = 1
    changed, c, o = oracle.majority_vote(pts, cams, masks)
    assert c.tolist() == [4, 1, 0] and o.tolist() == [0, 3, 4]
    assert changed.tolist() == [True, False, False]
    # thresholds: |I| < 2c is strict (c = 2 of 4: not changed; 3 of 4: changed)
    m2 = masks.copy()
    m2[2:, 24, 32] = 0
    assert oracle.majority_vote(pts[:, :1], cams, m2)[0].tolist() == [False]
    m2[2, 24, 32] = 1
    assert oracle.majority_vote(pts[:, :1], cams, m2)[0].tolist() == [True]
    # 4/3 o < |I|: (0, 0, -3.9) is outside three views (o = 3, 12 < 12 fails) and not
    # changed even with full masks
    p = np.array([[0.0], [0.0], [-3.9]])
    full = np.ones((4, 48, 64), np.uint8)
    ch, cc, oo = oracle.majority_vote(p, cams, full)
    assert oo.tolist() == [3] and cc.tolist() == [1] and ch.tolist() == [False]
    # with 200 px wide images cameras 1 and 3 see it too (u = 100 -+ 64 * 3.85 / 4): o = 1,
    # c = 3 -> changed; without the mask of one of them c = 2 -> not changed
    wide = scenes.ring_cameras(4, 4.0, width=200, height=48, fx=64.0)
    q = np.array([[0.0], [0.0], [-3.85]])
    full = np.ones((4, 48, 200), np.uint8)
    ch, cc, oo = oracle.majority_vote(q, wide, full)
    assert oo.tolist() == [1] and cc.tolist() == [3] and ch.tolist() == [True]
    full[1] = 0
    ch, cc, oo = oracle.majority_vote(q, wide, full)
    assert cc.tolist() == [2] and ch.tolist() == [False]
    # pixel boundaries: the origin lands exactly on u = 32.0, v = 24.0 -> pixel (32, 24)
    m3 = np.zeros((4, 48, 64), np.uint8)
    m3[:, 23, 31] = 1
    assert oracle.majority_vote(pts[:, :1], cams, m3)[1].tolist() == [0]

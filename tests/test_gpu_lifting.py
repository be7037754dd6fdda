"""Mask dilation and the majority vote on the GPU (clsp_dilate_masks,
clsp_majority_vote) against the CPU reference, bit for bit (Supp. "Detecting Changes in
2D"; Supp. "Identifying Changed 3D Regions via Majority Voting").

The change masks stand in for the paper's DINOv2 masks: the disk the change ball
projects to in each view (its centre's projection, radius f r / depth), dilated by 2%
of the width, as the benchmark's change masks are described."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_helpers import to_np
from paper_2506_21117_amd import api

pytestmark = pytest.mark.gpu


def _disk_masks(cams, center, radius):
    out = np.zeros((len(cams), cams[0].height, cams[0].width), np.uint8)
    for k, cam in enumerate(cams):
        p = np.asarray(cam.R, np.float64) @ np.asarray(center, np.float64) + np.asarray(cam.t, np.float64)
        if p[2] <= 0.2:
            continue
        u, v = cam.fx * p[0] / p[2] + cam.cx, cam.fy * p[1] / p[2] + cam.cy
        rr = cam.fx * radius / p[2]
        ys, xs = np.mgrid[0:cam.height, 0:cam.width]
        out[k] = ((xs + 0.5 - u) ** 2 + (ys + 0.5 - v) ** 2 <= rr * rr).astype(np.uint8)
    return out


@pytest.mark.parametrize("shape,radius,p", [((2, 37, 53), 4, 0.01), ((1, 720, 1280), 26, 2e-5),
                                             ((3, 19, 300), 0, 0.05), ((1, 21, 17), 40, 0.003),
                                             ((1, 1, 1), 2, 1.0)])
def test_dilation_bit_exact(dev, shape, radius, p):
    m = (np.random.default_rng(sum(shape) + radius).random(shape) < p).astype(np.uint8)
    got = api.dilate_masks(torch.as_tensor(m, device=dev), radius)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(to_np(got), oracle.dilate_masks(m, radius))


def test_dilated_disk_masks_of_the_benchmark_views(dev):
    w = scenes.local_change(n=1000, center=(0.0, 0.0, 1.0))
    masks = _disk_masks(w.cameras, (0.0, 0.0, 1.0), 0.4)
    r = api.dilation_radius(w.cameras[0].width)
    assert r == oracle.dilation_radius(w.cameras[0].width) == 26
    got = api.dilate_masks(torch.as_tensor(masks, device=dev), r)
    torch.cuda.synchronize()
    ref = oracle.dilate_masks(masks, r)
    np.testing.assert_array_equal(to_np(got), ref)
    assert ref.sum() > masks.sum() > 0


@pytest.mark.parametrize("center", [(0.0, 0.0, 0.0), (0.0, 0.0, 1.0)])
def test_majority_vote_bit_exact_at_full_size(dev, center):
    """The benchmark scene (10^6 Gaussians, 16 views of 1280x720) with the change ball's
    dilated disk masks: counts, decisions and their number equal the reference's; the
    vote selects most of the ball (every view sees the ball's disk, whatever occludes it)
    and few Gaussians far from it."""
    w = scenes.local_change(center=center)
    sc, cams = w.scene, w.cameras
    masks = oracle.dilate_masks(_disk_masks(cams, center, 0.4), oracle.dilation_radius(cams[0].width))
    means = torch.as_tensor(sc.means, device=dev)
    changed, cin, cout, cnt = api.majority_vote(means, cams, torch.as_tensor(masks, device=dev))
    torch.cuda.synchronize()
    ref_ch, ref_c, ref_o = oracle.majority_vote(sc.means, cams, masks)
    np.testing.assert_array_equal(to_np(cin).astype(np.int64), ref_c)
    np.testing.assert_array_equal(to_np(cout).astype(np.int64), ref_o)
    np.testing.assert_array_equal(to_np(changed).astype(bool), ref_ch)
    assert int(cnt.item()) == int(ref_ch.sum())
    d = np.linalg.norm(sc.means.astype(np.float64) - np.asarray(center)[:, None], axis=0)
    ball = np.zeros(sc.n, bool)
    ball[w.active_begin:] = True
    assert ref_ch[ball].mean() > 0.9
    assert ref_ch[d > 1.0].mean() < 0.01
    print(f"vote: {ref_ch.sum()} changed, {ref_ch[ball].mean():.3f} of the ball")

"""Pins of the change-region spheres in the CPU reference (Supp. "Identifying Changed 3D
Regions via Majority Voting": centre = cluster mean, radius = 1.1 x the 98th percentile
of the distances to it; Supp. "3DGS Optimization in Changed Regions": changed Gaussians
outside every sphere are removed), against values worked out by hand."""
import numpy as np

import oracle


def _shell(center, radius, pairs, rng):
    v = rng.normal(size=(3, pairs))
    v /= np.linalg.norm(v, axis=0)
    c = np.asarray(center, dtype=np.float64)[:, None]
    return np.concatenate([c + radius * v, c - radius * v], axis=1)     # symmetric: the mean is c


def test_sphere_of_a_shell_with_two_far_points():
    """98 points at distance 1 and 2 at distance 5 (symmetric pairs, mean exact):
    q = 0.98 * 99 = 97.02, sorted distances d[97] = 1, d[98] = 5, so the percentile is
    1 + 0.02 * 4 = 1.08 and the radius 1.188."""
    rng = np.random.default_rng(0)
    pts = np.concatenate([_shell((1, 2, 3), 1.0, 49, rng),
                          np.array([[6.0, -4.0], [2.0, 2.0], [3.0, 3.0]])], axis=1)
    c, r = oracle.fit_spheres(pts, np.zeros(100, int), 1)
    np.testing.assert_allclose(c[0], [1, 2, 3], atol=1e-13)
    assert abs(r[0] - 1.188) < 1e-12


def test_sphere_of_integer_distances_hits_an_order_statistic():
    """51 points at x = -25..25 on a line: distances 0, 1, 1, 2, 2, ..., 25, 25; q = 49
    exactly, d[49] = 25, radius 27.5.  A second cluster, points labelled -1 and an empty
    cluster in the same call."""
    xs = np.arange(-25, 26, dtype=np.float64)
    line = np.stack([xs + 10, np.zeros(51), np.zeros(51)])
    rng = np.random.default_rng(1)
    shell = _shell((-3, 0, 0), 2.0, 50, rng)
    noise = rng.normal(size=(3, 7)) * 100
    pts = np.concatenate([line, shell, noise], axis=1)
    labels = np.concatenate([np.zeros(51, int), np.full(100, 2), np.full(7, -1)])
    c, r = oracle.fit_spheres(pts, labels, 3)
    np.testing.assert_allclose(c[0], [10, 0, 0], atol=1e-12)
    assert abs(r[0] - 27.5) < 1e-12
    assert r[1] == -1.0 and np.all(c[1] == 0)
    np.testing.assert_allclose(c[2], [-3, 0, 0], atol=1e-13)
    assert abs(r[2] - 2.2) < 1e-12          # every distance is 2
    # one point: radius 0; two points: 1.1 x their common distance to the mean
    c1, r1 = oracle.fit_spheres(np.array([[1.0], [2.0], [3.0]]), [0], 1)
    assert r1[0] == 0.0 and np.all(c1[0] == [1, 2, 3])
    c2, r2 = oracle.fit_spheres(np.array([[0.0, 4.0], [0, 0], [0, 0]]), [0, 0], 1)
    assert c2[0][0] == 2.0 and abs(r2[0] - 2.2) < 1e-15


def test_membership_boundary_union_and_empty_spheres():
    centers = np.array([[0.0, 0.0, 0.0], [10.0, 0.0, 0.0], [0.0, 0.0, 0.0]])
    radii = np.array([2.0, 1.0, -1.0])
    f = np.float32
    pts = np.array([[2.0, 0.0, 0.0],                          # on the first sphere: inside
                    [np.nextafter(f(2.0), f(3.0)), 0.0, 0.0],  # one float32 step outside
                    [10.5, 0.5, 0.0],                          # in the second sphere only
                    [5.0, 0.0, 0.0],                           # in none
                    [0.0, 0.0, 0.0]]).T                        # centre (the empty sphere adds nothing)
    keep = oracle.sphere_keep(pts, centers, radii)
    assert keep.tolist() == [True, False, True, False, True]
    assert not oracle.sphere_keep(np.zeros((3, 1)), centers[2:], radii[2:])[0]


def test_compaction_keeps_the_static_prefix_and_the_order():
    a = np.arange(10, dtype=np.float32)
    b = np.arange(30, dtype=np.float32).reshape(3, 10)
    keep = np.array([True, False, True, True, False, False])          # rows 4..9
    na, nb = oracle.compact_rows([a, b], keep, 4)
    assert na.tolist() == [0, 1, 2, 3, 4, 6, 7]
    assert nb.tolist() == [[0, 1, 2, 3, 4, 6, 7], [10, 11, 12, 13, 14, 16, 17], [20, 21, 22, 23, 24, 26, 27]]

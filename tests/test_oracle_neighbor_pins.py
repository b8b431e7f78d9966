"""Pins of the oracle's neighbour search (the solver's use of the cell list, kernel
support 2h of Section 3): closed-form counts on perfect lattices, an independent
library (scipy's k-d tree), the strict inequality at the radius, and symmetry."""
import numpy as np
import pytest

import oracle


def _lattice(dim, n_side, dp=1.0):
    g = np.meshgrid(*[np.arange(n_side, dtype=np.float64) * dp] * dim, indexing="ij")
    pts = np.stack([a.ravel() for a in g], axis=1).astype(np.float32)
    return pts


@pytest.mark.parametrize("dim,radius,expect", [
    (2, 1.2, 4), (2, 1.5, 8), (2, 2.05, 12),          # shells 1, sqrt 2, 2
    (3, 1.2, 6), (3, 1.5, 18), (3, 1.8, 26),          # shells 1, sqrt 2, sqrt 3
])
def test_interior_lattice_counts(dim, radius, expect):
    pts = _lattice(dim, 7)
    z = pts[:, 2] if dim == 3 else None
    c = oracle.neighbor_count(dim, pts[:, 0], pts[:, 1], z, radius)
    interior = np.all((pts >= 3) & (pts <= 3), axis=1)  # the centre particle (3, 3[, 3])
    assert interior.sum() == 1
    assert c[interior][0] == expect
    # a corner particle of the 2-D lattice at radius 1.5 sees 3 (two faces, one diagonal)
    if dim == 2 and radius == 1.5:
        corner = np.all(pts == 0, axis=1)
        assert c[corner][0] == 3


def test_strict_inequality_at_the_radius():
    x = np.array([0.0, 0.5, 2.0], np.float32)
    y = np.zeros(3, np.float32)
    assert list(oracle.neighbor_count(2, x, y, None, 0.5)) == [0, 0, 0]      # exactly r apart: not neighbours
    r = np.nextafter(0.5, 1.0)
    assert list(oracle.neighbor_count(2, x, y, None, r)) == [1, 1, 0]


def test_against_scipy_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.Generator(np.random.PCG64(11))
    for dim in (2, 3):
        pts = rng.uniform(0.0, 1.0, size=(3000, dim)).astype(np.float32)
        r = 0.05 if dim == 2 else 0.11
        z = pts[:, 2] if dim == 3 else None
        c = oracle.neighbor_count(dim, pts[:, 0], pts[:, 1], z, r)
        tree = cKDTree(pts.astype(np.float64))
        ref = tree.query_ball_point(pts.astype(np.float64), r, return_length=True) - 1  # the point itself
        np.testing.assert_array_equal(c, ref)
        assert int(c.sum()) % 2 == 0                     # every pair is counted from both ends
        q = rng.choice(pts.shape[0], 50, replace=False)
        np.testing.assert_array_equal(oracle.neighbor_count(dim, pts[:, 0], pts[:, 1], z, r, query=q), c[q])

"""Pins for the Delaunay-by-lifting oracle: the empty-circle property by the
exact in-circle determinant (brute force), counter-clockwise triangles, the
count T = 2n - h - 2, and Qhull's (scipy) triangulation on points in general
position."""
import numpy as np
import pytest

from oracle import delaunay as dl
from oracle import validate


def general_position(rng, n, r=1 << 14):
    while True:
        p = rng.integers(-r, r, size=(n, 2), endpoint=True)
        if len({tuple(q) for q in p}) == n:
            return p.astype(np.int32)


def hull_vertex_count(p):
    import scipy.spatial
    return len(scipy.spatial.ConvexHull(p).vertices)


def test_empty_circles_and_orientation():
    rng = np.random.default_rng(8)
    for t in range(10):
        p = general_position(rng, int(rng.integers(4, 60)), 1 << 8)
        tris = dl.delaunay(p)
        assert all(o > 0 for o in dl.orient(p, tris))
        P = [tuple(int(v) for v in q) for q in p]
        for a, b, c in tris:
            for d in range(len(P)):
                if d not in (a, b, c):
                    assert dl.incircle(P, P[a], P[b], P[c], P[d]) <= 0
        assert len(tris) == 2 * len(p) - hull_vertex_count(p) - 2


def test_matches_qhull_in_general_position():
    import scipy.spatial
    rng = np.random.default_rng(9)
    for t in range(6):
        p = general_position(rng, 300)
        ours = validate.canonical(dl.delaunay(p))
        q = scipy.spatial.Delaunay(p.astype(np.float64)).simplices
        q = np.array([s if dl.orient(p, [s])[0] > 0 else s[[0, 2, 1]] for s in q])
        assert (ours == validate.canonical(q)).all()


def test_degenerate_grid():
    """A square grid: every unit square's four corners are cocircular and the
    boundary points are collinear.  The perturbation splits each unit square
    by one diagonal and adds zero-area triangles along the boundary; no point
    lies strictly inside any proper triangle's circle, and the triangles tile
    the rectangle exactly."""
    g = np.array([(x, y) for x in range(6) for y in range(5)], dtype=np.int32)
    tris = dl.delaunay(g)
    areas = dl.orient(g, tris)
    assert all(a >= 0 for a in areas) and sum(areas) == 2 * 5 * 4
    assert sum(1 for a in areas if a > 0) == 2 * 5 * 4  # two per unit square
    P = [tuple(int(v) for v in q) for q in g]
    for (a, b, c), ar in zip(tris, areas):
        if ar == 0:
            continue
        for d in range(len(P)):
            if d not in (a, b, c):
                assert dl.incircle(P, P[a], P[b], P[c], P[d]) <= 0


def test_full_range_general_position():
    """|x|, |y| up to 2^20 (lifted z up to 2^41): empty circles by the exact
    in-circle test, and Qhull's triangulation."""
    import scipy.spatial
    rng = np.random.default_rng(10)
    for t in range(3):
        p = general_position(rng, 40, 1 << 20)
        tris = dl.delaunay(p)
        assert all(o > 0 for o in dl.orient(p, tris))
        P = [tuple(int(v) for v in q) for q in p]
        for a, b, c in tris:
            for d in range(len(P)):
                if d not in (a, b, c):
                    assert dl.incircle(P, P[a], P[b], P[c], P[d]) <= 0
        assert len(tris) == 2 * len(p) - hull_vertex_count(p) - 2
    p = general_position(rng, 2000, 1 << 20)
    ours = validate.canonical(dl.delaunay(p))
    q = scipy.spatial.Delaunay(p.astype(np.float64)).simplices
    q = np.array([s if dl.orient(p, [s])[0] > 0 else s[[0, 2, 1]] for s in q])
    assert (ours == validate.canonical(q)).all()


def test_full_range_degenerate_grid():
    """The cocircular grid moved to the corner of the range: the same
    properties as at the origin (the split of each square may differ: the
    lifting turns a translation into a shear of z, which the perturbation of
    z does not follow, so only properties are compared)."""
    g = np.array([(x, y) for x in range(7) for y in range(6)], dtype=np.int64)
    g = g + np.array([(1 << 20) - 6, -(1 << 20)])
    tris = dl.delaunay(g)
    areas = dl.orient(g, tris)
    assert all(a >= 0 for a in areas) and sum(areas) == 2 * 6 * 5
    assert sum(1 for a in areas if a > 0) == 2 * 6 * 5
    P = [tuple(int(v) for v in q) for q in g]
    for (a, b, c), ar in zip(tris, areas):
        if ar == 0:
            continue
        for d in range(len(P)):
            if d not in (a, b, c):
                assert dl.incircle(P, P[a], P[b], P[c], P[d]) <= 0
    with pytest.raises(ValueError):
        dl.delaunay(np.array([[0, 0], [1, 0], [(1 << 20) + 1, 5]]))

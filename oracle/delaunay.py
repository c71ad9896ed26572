"""2-d Delaunay triangulation by lifting (test infrastructure): the lower
hull of (x, y, x^2 + y^2) under the oracle's perturbed exact hull (its wide
range: |x|, |y| <= 2^20, lifted z <= 2^41), each lower face turned
counter-clockwise in the plane.  Plus the checks that pin
it: the exact in-circle test and the triangle count."""
import numpy as np

from . import hull_wide as _hull_wide


MAX_XY = 1 << 20  # lifted z = x^2 + y^2 <= 2^41: the oracle's wide range


def lift(xy):
    xy = np.asarray(xy, dtype=np.int64).reshape(-1, 2)
    z = xy[:, 0] * xy[:, 0] + xy[:, 1] * xy[:, 1]
    return np.ascontiguousarray(np.column_stack([xy, z]))


def delaunay(xy):
    """Triangles [T, 3] of input indices, counter-clockwise (|x|, |y| <=
    2^20)."""
    xy = np.asarray(xy).reshape(-1, 2)
    if np.abs(xy).max(initial=0) > MAX_XY:
        raise ValueError("|x|, |y| must be at most 2^20")
    if len(xy) < 3:
        return np.zeros((0, 3), dtype=np.int32)
    f = _hull_wide(lift(xy), lower_only=True)
    return np.ascontiguousarray(f[:, [0, 2, 1]]).astype(np.int32)


def orient(xy, t):
    """Twice the signed area of each triangle (exact, Python integers)."""
    p = [[int(v) for v in r] for r in np.asarray(xy)]
    out = []
    for a, b, c in np.asarray(t):
        (ax, ay), (bx, by), (cx, cy) = p[a], p[b], p[c]
        out.append((bx - ax) * (cy - ay) - (cx - ax) * (by - ay))
    return out


def incircle(p, a, b, c, d):
    """> 0 when d lies strictly inside the circle through the counter-
    clockwise triangle (a, b, c) (exact determinant, Python integers)."""
    rows = []
    for q in (a, b, c):
        dx, dy = q[0] - d[0], q[1] - d[1]
        rows.append((dx, dy, dx * dx + dy * dy))
    (a1, a2, a3), (b1, b2, b3), (c1, c2, c3) = rows
    return (a1 * (b2 * c3 - b3 * c2) - a2 * (b1 * c3 - b3 * c1) + a3 * (b1 * c2 - b2 * c1))

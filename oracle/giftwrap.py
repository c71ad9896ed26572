"""3-d gift wrapping under the same symbolic perturbation (test
infrastructure): an algorithm independent of the kinetic method, used to check
the oracle on inputs too large for brute force.

Starting from one hull face, every face edge (a, b) is wrapped: the neighbour
face is (b, a, r) for the point r that leaves every other point on the inner
side, i.e. the maximum of the rotation order around the edge, where r2 beats
r1 when orient(b, a, r1, r2) > 0.  All points lie in the closed half-space of
the current face, so this order is a strict total order and a pairwise
tournament finds its maximum.
"""
import numpy as np

from .brute import _SUBSETS


class _Orient:
    def __init__(self, P, I):
        P = np.asarray(P, dtype=np.int64)
        I = np.asarray(I, dtype=np.int64)
        cb = int(np.abs(P).max(initial=0)).bit_length() + 1
        ib = int(np.max(I, initial=0)).bit_length()
        if 2 * cb + 3 * ib + 3 > 62 or cb + 5 * ib + 3 > 62 or 6 * ib + 3 > 62:
            raise ValueError("gift-wrap needs small coordinates and indices (int64 exactness)")
        self.base = [P[:, 0], P[:, 1], P[:, 2]]
        self.pert = [I, I * I, I * I * I]

    def sign(self, a, b, c, d):
        """Perturbed orientation sign of (a, b, c, d), vectorised over arrays."""
        a, b, c, d = (np.asarray(q, dtype=np.int64) for q in (a, b, c, d))
        shape = np.broadcast(a, b, c, d).shape
        sg = np.zeros(shape, dtype=np.int8)
        for S in _SUBSETS:
            col = [self.pert[k] if k in S else self.base[k] for k in range(3)]
            u = [col[k][b] - col[k][a] for k in range(3)]
            v = [col[k][c] - col[k][a] for k in range(3)]
            w = [col[k][d] - col[k][a] for k in range(3)]
            det = (u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0])
                   + u[2] * (v[0] * w[1] - v[1] * w[0]))
            sg = np.where(sg == 0, np.sign(det).astype(np.int8), sg)
        return sg

    def dsign(self, a, b, c):
        """Perturbed sign of the xy orientation D(a, b, c), vectorised."""
        a, b, c = (np.asarray(q, dtype=np.int64) for q in (a, b, c))
        sg = np.zeros(np.broadcast(a, b, c).shape, dtype=np.int8)
        for S in [(), (0,), (1,), (0, 1)]:
            col = [self.pert[k] if k in S else self.base[k] for k in range(2)]
            det = ((col[0][b] - col[0][a]) * (col[1][c] - col[1][a])
                   - (col[0][c] - col[0][a]) * (col[1][b] - col[1][a]))
            sg = np.where(sg == 0, np.sign(det).astype(np.int8), sg)
        return sg


def _is_face(O, n, a, b, c):
    d = np.array([q for q in range(n) if q not in (a, b, c)], dtype=np.int64)
    s = O.sign(a, b, c, d)
    return bool((s < 0).all())


def _wrap(O, n, a, b):
    """Point r making (b, a, r) a face, given that edge (a, b) is on the hull."""
    cand = np.array([q for q in range(n) if q != a and q != b], dtype=np.int64)
    while len(cand) > 1:
        if len(cand) % 2:
            odd, cand = cand[-1:], cand[:-1]
        else:
            odd = cand[:0]
        r1, r2 = cand[0::2], cand[1::2]
        s = O.sign(b, a, r1, r2)
        cand = np.concatenate([np.where(s > 0, r2, r1), odd])
    return int(cand[0])


def hull_faces(P, I=None):
    """Outward faces (positions into P) by gift wrapping."""
    P = np.asarray(P, dtype=np.int64).reshape(-1, 3)
    n = len(P)
    I = np.arange(n, dtype=np.int64) if I is None else np.asarray(I, dtype=np.int64)
    if n < 3:
        return np.zeros((0, 3), dtype=np.int64)
    if n == 3:
        return np.array([[0, 1, 2], [0, 2, 1]], dtype=np.int64)
    O = _Orient(P, I)
    # A first edge: p0, the x-extreme point (smallest (x, index)), and q, its
    # clockwise neighbour on the hull of the xy-projection (every other point
    # strictly left of p0 -> q).  The vertical plane through p0 and q
    # supports the set, so p0-q is a hull edge.
    p0 = int(np.lexsort((I, P[:, 0]))[0])
    cand = np.array([q for q in range(n) if q != p0], dtype=np.int64)
    while len(cand) > 1:
        if len(cand) % 2:
            odd, cand = cand[-1:], cand[:-1]
        else:
            odd = cand[:0]
        r1, r2 = cand[0::2], cand[1::2]
        s = O.dsign(p0, r1, r2)
        cand = np.concatenate([np.where(s < 0, r2, r1), odd])
    q = int(cand[0])
    # One of the two faces on that edge: (q, p0, r) with r wrapped around it.
    r = _wrap(O, n, p0, q)
    first = (q, p0, r)
    assert _is_face(O, n, *first)
    first = min([first, (first[1], first[2], first[0]), (first[2], first[0], first[1])])
    faces = {first}
    todo = [first]
    done_edges = set()
    while todo:
        f = todo.pop()
        for a, b in ((f[0], f[1]), (f[1], f[2]), (f[2], f[0])):
            if (b, a) in done_edges:
                continue
            r = _wrap(O, n, a, b)
            g = (b, a, r)
            # rotate to the canonical start so duplicates are recognised
            rots = [g, (g[1], g[2], g[0]), (g[2], g[0], g[1])]
            g = min(rots)
            for x, y in ((g[0], g[1]), (g[1], g[2]), (g[2], g[0])):
                done_edges.add((x, y))
            done_edges.add((a, b))
            if g not in faces:
                faces.add(g)
                todo.append(g)
    return np.array(sorted(faces), dtype=np.int64)

"""O(n^4) brute-force hull and block movies under the symbolic perturbation
(test infrastructure; the plain definition of the result).

A triple of points is a face of the hull of the perturbed points exactly when
every other point lies strictly on one side of its plane (the perturbation
makes every orientation nonzero).  The orientation det[b~-a~; c~-a~; d~-a~] of
perturbed points p~ = (x + e1*i, y + e2*i^2, z + e3*i^3) is multilinear in its
columns, so its coefficient for a set S of columns is the same determinant
with the columns in S replaced by the index-power differences; the monomials
1, e1, e2, e1e2, e3, e1e3, e2e3, e1e2e3 are in decreasing order of size.
That expansion is evaluated here in numpy int64 (inputs are kept small enough
to be exact) and is itself pinned by ``perturb`` in the tests.

The movie of a block (Sec. 2: the time-ordered event list of the kinetic 2-d
hull) is, by the kinetic model, its lower faces sorted by event time
tau = N / D, each face an event of its middle vertex in x-order.
"""
from itertools import combinations

import numpy as np

from . import perturb

# Column subsets in decreasing monomial size: 1, e1, e2, e1e2, e3, e1e3, e2e3, e1e2e3.
_SUBSETS = [(), (0,), (1,), (0, 1), (2,), (0, 2), (1, 2), (0, 1, 2)]


def _check_small(P, I):
    cb = int(np.abs(P).max(initial=0)).bit_length() + 1
    ib = int(np.max(I, initial=0)).bit_length()
    if 2 * cb + 3 * ib + 3 > 62 or cb + 2 * ib + 3 * ib + 3 > 62 or 6 * ib + 3 > 62:
        raise ValueError("brute force needs small coordinates and indices (int64 exactness)")


def rank_order(P, I):
    """Ranks by (x, index): the x-order of the perturbed points."""
    return np.lexsort((I, P[:, 0]))


def orient3d_signs(P, I, A, B, C):
    """Perturbed orientation sign of (A[t], B[t], C[t], d) for every triple t
    and every point d: int8 array [T, n]; 0 where d is one of the triple."""
    P = np.asarray(P, dtype=np.int64)
    I = np.asarray(I, dtype=np.int64)
    base = [P[:, 0], P[:, 1], P[:, 2]]
    pert = [I, I * I, I * I * I]
    T, n = len(A), len(P)
    sg = np.zeros((T, n), dtype=np.int8)
    for S in _SUBSETS:
        c = [pert[k] if k in S else base[k] for k in range(3)]
        u = [c[k][B] - c[k][A] for k in range(3)]
        v = [c[k][C] - c[k][A] for k in range(3)]
        w = [c[k][None, :] - c[k][A][:, None] for k in range(3)]
        det = (u[0][:, None] * (v[1][:, None] * w[2] - v[2][:, None] * w[1])
               - u[1][:, None] * (v[0][:, None] * w[2] - v[2][:, None] * w[0])
               + u[2][:, None] * (v[0][:, None] * w[1] - v[1][:, None] * w[0]))
        s = np.sign(det).astype(np.int8)
        sg = np.where(sg == 0, s, sg)
    rows = np.arange(T)
    sg[rows, A] = 0
    sg[rows, B] = 0
    sg[rows, C] = 0
    return sg


def d_sign(P, I, a, b, c):
    """Perturbed sign of D(a, b, c), the z-component of (b~-a~) x (c~-a~)."""
    P = np.asarray(P, dtype=np.int64)
    I = np.asarray(I, dtype=np.int64)
    base = [P[:, 0], P[:, 1]]
    pert = [I, I * I]
    for S in [(), (0,), (1,), (0, 1)]:
        c2 = [pert[k] if k in S else base[k] for k in range(2)]
        v = ((c2[0][b] - c2[0][a]) * (c2[1][c] - c2[1][a])
             - (c2[0][c] - c2[0][a]) * (c2[1][b] - c2[1][a]))
        if v != 0:
            return int(np.sign(v))
    raise AssertionError("D vanished for distinct indices")


def hull_faces(P, I=None, chunk=20000):
    """All outward faces of the perturbed hull, as triples of positions into P."""
    P = np.asarray(P, dtype=np.int64).reshape(-1, 3)
    n = len(P)
    I = np.arange(n, dtype=np.int64) if I is None else np.asarray(I, dtype=np.int64)
    _check_small(P, I)
    if n < 3:
        return np.zeros((0, 3), dtype=np.int64)
    if n == 3:
        return np.array([[0, 1, 2], [0, 2, 1]], dtype=np.int64)
    tri = np.array(list(combinations(range(n), 3)), dtype=np.int64)
    out = []
    for s in range(0, len(tri), chunk):
        t = tri[s: s + chunk]
        sg = orient3d_signs(P, I, t[:, 0], t[:, 1], t[:, 2])
        neg = (sg <= 0).all(axis=1)
        pos = (sg >= 0).all(axis=1)
        for r in np.nonzero(neg)[0]:
            out.append(t[r])
        for r in np.nonzero(pos)[0]:
            out.append(t[r][[0, 2, 1]])
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def split_lower_upper(P, I, faces):
    """Lower faces have outward normal with negative (perturbed) z."""
    lo, up = [], []
    for f in faces:
        (lo if d_sign(P, I, f[0], f[1], f[2]) < 0 else up).append(f)
    return np.array(lo, dtype=np.int64).reshape(-1, 3), np.array(up, dtype=np.int64).reshape(-1, 3)


def block_movie(P, I, ranks, run):
    """Movie of the block made of the points ``ranks`` (rank order) for run 0
    (lower) or 1 (upper): events (left, middle, right, is_insertion) in ranks,
    sorted by (event time, rank triple)."""
    ranks = np.asarray(ranks, dtype=np.int64)
    sub_P = np.asarray(P, dtype=np.int64)[ranks]
    sub_I = np.asarray(I, dtype=np.int64)[ranks]
    if len(ranks) < 3:
        return np.zeros((0, 4), dtype=np.int64)
    faces = hull_faces(sub_P, sub_I)
    K = perturb.choose_k(np.abs(sub_P).max(), sub_I.max())
    pz = perturb.Perturbed(sub_P, sub_I, K, zsign=1 if run == 0 else -1)
    ev = []
    for f in faces:
        if run == 0 and d_sign(sub_P, sub_I, *f) >= 0:
            continue
        if run == 1 and d_sign(sub_P, sub_I, *f) <= 0:
            continue
        l, m, r = sorted(int(q) for q in f)  # positions in the block = rank order
        tau = pz.tau(l, m, r)
        ins = 1 if d_sign(sub_P, sub_I, l, m, r) < 0 else 0
        ev.append((tau, (int(ranks[l]), int(ranks[m]), int(ranks[r])), ins))
    ev.sort(key=lambda e: (e[0], e[1]))
    return np.array([[*e[1], e[2]] for e in ev], dtype=np.int64).reshape(-1, 4)


def hull_faces_exact(P, I=None):
    """hull_faces for any coordinate size (tiny n): every orientation is the
    textbook determinant of points moved by concrete tiny epsilons, in exact
    big integers (``perturb``)."""
    P = [[int(v) for v in r] for r in np.asarray(P).reshape(-1, 3)]
    n = len(P)
    I = list(range(n)) if I is None else [int(i) for i in I]
    if n < 3:
        return np.zeros((0, 3), dtype=np.int64)
    if n == 3:
        return np.array([[0, 1, 2], [0, 2, 1]], dtype=np.int64)
    K = perturb.choose_k(max(abs(v) for r in P for v in r), max(I))
    pz = perturb.Perturbed(P, I, K)
    out = []
    for a, b, c in combinations(range(n), 3):
        sg = [perturb.sign(pz.orient3d(a, b, c, d)) for d in range(n) if d not in (a, b, c)]
        if all(v < 0 for v in sg):
            out.append((a, b, c))
        elif all(v > 0 for v in sg):
            out.append((a, c, b))
    return np.array(out, dtype=np.int64).reshape(-1, 3)

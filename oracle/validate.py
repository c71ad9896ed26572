"""Structural checks on a face list (test infrastructure).

canonical   rotate each triple so its smallest index comes first (keeping the
            orientation) and sort the rows: the form in which two face sets
            are compared.
euler_ok    a simplicial closed convex surface on V vertices has F = 2V - 4.
manifold_ok every directed edge appears exactly once, and so does its reverse.
containment every input point lies on or inside every face's plane (exact
            orient3d on the unperturbed integers, a float filter with an exact
            big-integer fallback).
"""
import numpy as np


def canonical(faces):
    f = np.asarray(faces, dtype=np.int64).reshape(-1, 3)
    if len(f) == 0:
        return f.copy()
    k = np.argmin(f, axis=1)
    rows = np.arange(len(f))
    g = np.stack([f[rows, k], f[rows, (k + 1) % 3], f[rows, (k + 2) % 3]], axis=1)
    order = np.lexsort((g[:, 2], g[:, 1], g[:, 0]))
    return g[order]


def vertex_count(faces):
    return len(np.unique(np.asarray(faces).reshape(-1))) if len(faces) else 0


def euler_ok(faces):
    f = np.asarray(faces).reshape(-1, 3)
    if len(f) == 0:
        return True
    return len(f) == 2 * vertex_count(f) - 4


def manifold_ok(faces):
    f = np.asarray(faces, dtype=np.int64).reshape(-1, 3)
    if len(f) == 0:
        return True
    a = np.concatenate([f[:, 0], f[:, 1], f[:, 2]])
    b = np.concatenate([f[:, 1], f[:, 2], f[:, 0]])
    m = int(max(a.max(), b.max())) + 1
    key = a * m + b
    rkey = b * m + a
    if len(np.unique(key)) != len(key):
        return False
    return bool(np.isin(rkey, key).all())


def _orient_exact(p, q, r, s):
    u = [int(q[k]) - int(p[k]) for k in range(3)]
    v = [int(r[k]) - int(p[k]) for k in range(3)]
    w = [int(s[k]) - int(p[k]) for k in range(3)]
    return (u[0] * (v[1] * w[2] - v[2] * w[1]) - u[1] * (v[0] * w[2] - v[2] * w[0])
            + u[2] * (v[0] * w[1] - v[1] * w[0]))


def containment_violations(P, faces, points=None, chunk=1 << 22):
    """Number of (face, point) pairs with the point strictly outside the
    face's plane.  ``points`` optionally restricts the points checked."""
    P = np.asarray(P, dtype=np.int64).reshape(-1, 3)
    f = np.asarray(faces, dtype=np.int64).reshape(-1, 3)
    Q = P if points is None else P[np.asarray(points)]
    Pf = P.astype(np.float64)
    Qf = Q.astype(np.float64)
    bad = 0
    fstep = max(1, chunk // max(len(Q), 1))
    for s in range(0, len(f), fstep):
        ff = f[s: s + fstep]
        a, b, c = Pf[ff[:, 0]], Pf[ff[:, 1]], Pf[ff[:, 2]]
        u = b - a
        v = c - a
        w = Qf[None, :, :] - a[:, None, :]
        m0 = u[:, 1] * v[:, 2] - u[:, 2] * v[:, 1]
        m1 = u[:, 2] * v[:, 0] - u[:, 0] * v[:, 2]
        m2 = u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0]
        det = m0[:, None] * w[:, :, 0] + m1[:, None] * w[:, :, 1] + m2[:, None] * w[:, :, 2]
        perm = ((np.abs(u[:, 1] * v[:, 2]) + np.abs(u[:, 2] * v[:, 1]))[:, None] * np.abs(w[:, :, 0])
                + (np.abs(u[:, 2] * v[:, 0]) + np.abs(u[:, 0] * v[:, 2]))[:, None] * np.abs(w[:, :, 1])
                + (np.abs(u[:, 0] * v[:, 1]) + np.abs(u[:, 1] * v[:, 0]))[:, None] * np.abs(w[:, :, 2]))
        tol = 1e-14 * perm
        bad += int((det > tol).sum())
        amb = np.nonzero(np.abs(det) <= tol)
        for i, j in zip(*amb):
            fi = ff[i]
            if _orient_exact(P[fi[0]], P[fi[1]], P[fi[2]], Q[j]) > 0:
                bad += 1
    return bad

"""FP64 volume, surface area and their gradients of a closed triangulated
surface (test infrastructure; the plain definition written out in numpy).

For outward faces (a, b, d) of a closed surface and any reference point c:
    V = 1/6 sum_f (a - c) . ((b - c) x (d - c))
    A = 1/2 sum_f |(b - a) x (d - a)|
The reference point used here is the cloud's point 0 (any point gives the same
V on a closed surface; a point of the cloud lies in its hull, so every term
is non-negative).  Gradients with respect to the positions, on the fixed face
set: for a vertex a and each face f = (a, b, d) rotated to start at a,
    dV/da = 1/6 sum_f (b - a) x (d - a)     (the reference point cancels)
    dA/da = 1/2 sum_f (b - d) x n_f,   n_f = unit normal of (b - a) x (d - a)
(zero for faces of zero area).
"""
import numpy as np


def volume_area(P, faces):
    P = np.asarray(P, dtype=np.float64)
    f = np.asarray(faces, dtype=np.int64).reshape(-1, 3)
    if len(f) == 0:
        return 0.0, 0.0
    c = P[0]
    a, b, d = P[f[:, 0]], P[f[:, 1]], P[f[:, 2]]
    V = np.sum(np.einsum("ij,ij->i", a - c, np.cross(b - c, d - c))) / 6.0
    A = 0.5 * np.sum(np.linalg.norm(np.cross(b - a, d - a), axis=1))
    return float(V), float(A)


def gradients(P, faces):
    """(dV/dP, dA/dP), each [n, 3] float64."""
    P = np.asarray(P, dtype=np.float64)
    f = np.asarray(faces, dtype=np.int64).reshape(-1, 3)
    gV = np.zeros_like(P)
    gA = np.zeros_like(P)
    for rot in range(3):
        ia, ib, id_ = f[:, rot], f[:, (rot + 1) % 3], f[:, (rot + 2) % 3]
        a, b, d = P[ia], P[ib], P[id_]
        n = np.cross(b - a, d - a)
        nn = np.linalg.norm(n, axis=1, keepdims=True)
        nhat = np.divide(n, nn, out=np.zeros_like(n), where=nn > 0)
        np.add.at(gV, ia, n / 6.0)
        np.add.at(gA, ia, 0.5 * np.cross(b - d, nhat))
    return gV, gA


def finite_difference(P, faces, coords, h=1.0):
    """Central differences of (V, A) at the (point, axis) pairs in coords."""
    P = np.asarray(P, dtype=np.float64)
    out = []
    for (i, k) in coords:
        Q = P.copy()
        Q[i, k] += h
        Vp, Ap = volume_area(Q, faces)
        Q[i, k] -= 2 * h
        Vm, Am = volume_area(Q, faces)
        out.append(((Vp - Vm) / (2 * h), (Ap - Am) / (2 * h)))
    return np.array(out)

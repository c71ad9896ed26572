"""Pins for the FP64 volume/area oracle: closed forms, exact identities of
the gradients, and central finite differences (V is linear in each
coordinate, so its central difference is exact up to rounding)."""
import numpy as np

import oracle
from oracle import volume_area as va
from paper_1205_1171_amd import workloads


def test_closed_forms():
    cube = workloads.cube_corners(1).astype(np.float64)
    f = oracle.hull(workloads.cube_corners(1))
    V, A = va.volume_area(cube, f)
    assert abs(V - 1.0) < 1e-15 and abs(A - 6.0) < 1e-14
    tet = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    f = oracle.hull(tet.astype(np.int32))
    V, A = va.volume_area(tet, f)
    assert abs(V - 1 / 6) < 1e-15
    assert abs(A - (1.5 + np.sqrt(3) / 2)) < 1e-14
    oc = workloads.octahedron(3).astype(np.float64)
    V, A = va.volume_area(oc, oracle.hull(workloads.octahedron(3)))
    assert abs(V - 4 / 3 * 27) < 1e-12  # |x|+|y|+|z| <= 3: (4/3) r^3
    assert abs(A - 8 * np.sqrt(3) / 4 * 18) < 1e-11  # 8 equilateral faces, side 3*sqrt(2)


def _cloud(seed, m=400):
    rng = np.random.default_rng(seed)
    P = workloads.noisy_sphere(rng, m, radius=float(1 << 10), sigma=8.0)
    Q = np.rint(P).astype(np.int32)
    f = oracle.hull(Q)
    return P.astype(np.float64), f


def test_identities():
    for seed in range(4):
        P, f = _cloud(seed)
        V, A = va.volume_area(P, f)
        gV, gA = va.gradients(P, f)
        scale_v, scale_a = np.abs(P).max() * np.abs(gV).max(), np.abs(P).max() * np.abs(gA).max()
        # translation invariance
        assert np.allclose(gV.sum(axis=0), 0, atol=1e-9 * scale_v)
        assert np.allclose(gA.sum(axis=0), 0, atol=1e-9 * scale_a)
        # homogeneity: V of degree 3, A of degree 2
        assert abs((P * gV).sum() - 3 * V) < 1e-9 * abs(V)
        assert abs((P * gA).sum() - 2 * A) < 1e-9 * abs(A)
        # rotation invariance
        assert np.allclose(np.cross(P, gV).sum(axis=0), 0, atol=1e-9 * scale_v)
        # the reference point does not matter on a closed surface
        Vs, _ = va.volume_area(P + 123.0, f)
        assert abs(Vs - V) < 1e-9 * V


def test_finite_differences():
    for seed in range(3):
        P, f = _cloud(seed + 10)
        gV, gA = va.gradients(P, f)
        rng = np.random.default_rng(seed)
        verts = np.unique(f)
        coords = [(int(rng.choice(verts)), int(rng.integers(0, 3))) for _ in range(40)]
        fd = va.finite_difference(P, f, coords, h=1e-3)
        an = np.array([[gV[i, k], gA[i, k]] for i, k in coords])
        assert np.linalg.norm(fd[:, 0] - an[:, 0]) <= 1e-7 * np.linalg.norm(an[:, 0])
        assert np.linalg.norm(fd[:, 1] - an[:, 1]) <= 1e-6 * np.linalg.norm(an[:, 1])

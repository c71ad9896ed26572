"""Pins of the oracle on its wide range (|x|, |y| <= 2^30, |z| <= 2^42) and of
the float-input snap (CPU).

The wide entry runs the same method as the int32 one on int64 rows; what is
new is the size of every intermediate, so the pins exercise large values:
  * brute force with exact big-integer orientations at concrete tiny
    epsilons, on tiny inputs spread over the whole wide range;
  * invariance: scaling every coordinate by a positive power of two, or
    translating all points, changes no predicate's sign (each epsilon
    coefficient of D, N and of the time comparison scales by one positive
    factor; translations cancel in differences), so the face set of a
    narrow input must come out of the wide entry unchanged;
  * scipy's Qhull on points in general position at the wide range;
  * the float snap against the same scale-and-round done in exact rationals.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute, floatin, validate
from paper_1205_1171_amd import workloads

XY, Z = 1 << 30, 1 << 42


def _same(a, b):
    a, b = validate.canonical(a), validate.canonical(b)
    return a.shape == b.shape and bool((a == b).all())


def test_wide_matches_exact_brute_force():
    rng = np.random.default_rng(41)
    for t in range(36):
        n = int(rng.integers(4, 11))
        if t % 3 == 0:     # random over the whole range
            p = np.column_stack([rng.integers(-XY, XY, n, endpoint=True),
                                 rng.integers(-XY, XY, n, endpoint=True),
                                 rng.integers(-Z, Z, n, endpoint=True)])
        elif t % 3 == 1:   # a degenerate lattice, scaled up and moved to the corner
            q = rng.integers(0, 3, size=(n, 3), endpoint=True)
            p = q * np.array([1 << 27, 1 << 27, 1 << 39]) + np.array([XY - (3 << 27), -XY, Z - (3 << 39)])
        else:              # near-coplanar large values and duplicates
            q = rng.integers(-5, 5, size=(n, 3), endpoint=True)
            p = q + np.array([XY - 8, XY - 8, -Z + 8])
            p[n // 2:] = p[: n - n // 2]
        got = oracle.hull_wide(p)
        want = brute.hull_faces_exact(p)
        assert _same(got, want), t


@pytest.mark.parametrize("kind", ["lattice", "cube", "flatx"])
def test_scale_and_translation_invariance(kind):
    rng = np.random.default_rng(42)
    for t in range(6):
        n = int(rng.integers(20, 400))
        if kind == "lattice":
            p = workloads.lattice(rng, n, 6).astype(np.int64)
        elif kind == "cube":
            p = workloads.cube(rng, n, 1 << 10).astype(np.int64)
        else:
            p = workloads.lattice(rng, n, 9).astype(np.int64)
            p[:, 0] = 2
        want = oracle.hull(p.astype(np.int32))
        assert _same(oracle.hull_wide(p), want)
        assert _same(oracle.hull_wide(p << 19), want)   # scaled by 2^19
        shift = np.array([XY - 2048, -XY + 2048, Z - 4096])
        assert _same(oracle.hull_wide(p + shift), want)
        assert _same(oracle.hull_wide(p, lower_only=True), oracle.hull(p.astype(np.int32), lower_only=True))


def test_wide_matches_qhull_general_position():
    from scipy.spatial import ConvexHull
    rng = np.random.default_rng(43)
    for t in range(4):
        n = 400
        p = np.column_stack([rng.integers(-XY, XY, n, endpoint=True),
                             rng.integers(-XY, XY, n, endpoint=True),
                             rng.integers(-Z, Z, n, endpoint=True)])
        f = oracle.hull_wide(p)
        h = ConvexHull(p.astype(np.float64))
        a = {tuple(sorted(r)) for r in f.tolist()}
        b = {tuple(sorted(r)) for r in h.simplices.tolist()}
        assert a == b
        assert validate.euler_ok(f) and validate.manifold_ok(f)


def test_wide_rejects_out_of_range():
    p = np.array([[0, 0, 0], [1, 1, 1], [XY + 1, 0, 0]])
    with pytest.raises(oracle.OracleError):
        oracle.hull_wide(p)
    p = np.array([[0, 0, 0], [1, 1, 1], [0, 0, Z + 1]])
    with pytest.raises(oracle.OracleError):
        oracle.hull_wide(p)


def _lattice_exact(p32, bits):
    """The snap in exact rationals: E from the largest magnitude, then
    round half to even of c * 2^(bits - E)."""
    vals = [Fraction(float(v)) for v in np.asarray(p32, dtype=np.float32).reshape(-1)]
    m = max(abs(v) for v in vals)
    E = 0
    if m > 0:
        while Fraction(2) ** E < m:
            E += 1
        while Fraction(2) ** (E - 1) >= m:
            E -= 1
    s = Fraction(2) ** (bits - E)
    out = []
    for v in vals:
        x = v * s
        fl = x.numerator // x.denominator
        r = x - fl
        q = fl + (1 if r > Fraction(1, 2) or (r == Fraction(1, 2) and fl % 2 == 1) else 0)
        out.append(q)
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def test_float_snap_exact():
    rng = np.random.default_rng(44)
    cases = [rng.standard_normal((50, 3)).astype(np.float32) * 1000,
             (rng.random((50, 3)) * 1e-30).astype(np.float32),
             np.ldexp(rng.integers(-8, 8, size=(40, 3)), 5).astype(np.float32),   # max 2^8 exactly
             rng.uniform(-3e38, 3e38, size=(30, 3)).astype(np.float32),
             np.array([[0.5, -0.25, 0.0], [1.5, 2.5, -3.5]], np.float32),          # halves round to even
             np.zeros((4, 3), np.float32)]
    for p in cases:
        for bits in (1, 5, 20, 29, 30):
            q = floatin.lattice(p, bits)
            assert (q == _lattice_exact(p, bits)).all()
            assert np.abs(q).max(initial=0) <= 1 << bits
    # floats within 2^(bits - 23) of the largest magnitude are kept exactly
    p = np.array([[1.0, 3.0, 0.75], [5.0, -7.0, 8.0]], np.float32)
    q = floatin.lattice(p, 30)
    assert (q == (p.astype(np.float64) * 2 ** 27).astype(np.int64)).all()
    with pytest.raises(ValueError):
        floatin.lattice(np.array([[np.inf, 0, 0]], np.float32), 30)


def test_float_hull_is_lattice_hull():
    """The float path's hull is the integer hull of the snapped points."""
    rng = np.random.default_rng(45)
    p = (workloads.sphere(rng, 2000, 1 << 20).astype(np.float32) * 1.37e-3).astype(np.float32)
    for bits in (20, 29):
        want = oracle.hull(floatin.lattice(p, bits).astype(np.int32))
        assert _same(floatin.hull_f32(p, bits), want)
    f = floatin.hull_f32(p, 30)
    assert validate.euler_ok(f) and validate.manifold_ok(f)

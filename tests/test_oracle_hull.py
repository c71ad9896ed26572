"""Pins for the oracle's hull, movies and chains.

Against: the O(n^4) brute-force definition (exact face-set equality, many
small and heavily degenerate inputs), an independent gift-wrap, scipy's Qhull
on general-position inputs, closed forms (tetrahedron, octahedron, cube,
cyclic polytope by Gale's evenness condition), and structural invariants
(Euler count, closed 2-manifold, containment, movie size bounds, the -inf
chain as a 2-d monotone-chain lower hull).
"""
import numpy as np
import pytest

import oracle
from oracle import brute, giftwrap, validate
from paper_1205_1171_amd import workloads


def same(a, b):
    a = validate.canonical(a)
    b = validate.canonical(b)
    return a.shape == b.shape and bool((a == b).all())


def _degenerate_cases(rng, count):
    for t in range(count):
        n = int(rng.integers(3, 30))
        kind = t % 8
        if kind == 0:
            p = workloads.lattice(rng, n, 1)
        elif kind == 1:
            p = workloads.lattice(rng, n, 2)
        elif kind == 2:
            p = workloads.lattice(rng, n, 3)
        elif kind == 3:
            p = workloads.lattice(rng, n, 7)
        elif kind == 4:  # one x value: the planar blocks of the Gaussian workload
            p = workloads.lattice(rng, n, 5)
            p[:, 0] = 2
        elif kind == 5:  # one z value
            p = workloads.lattice(rng, n, 5)
            p[:, 2] = -1
        elif kind == 6:  # many duplicates
            q = workloads.lattice(rng, max(n // 3, 1), 4)
            p = q[rng.integers(0, len(q), size=n)]
        else:
            p = rng.integers(-1000, 1001, size=(n, 3)).astype(np.int32)
        yield p


def test_matches_brute_force_degenerate(rng):
    for p in _degenerate_cases(rng, 400):
        want = brute.hull_faces(p)
        assert same(oracle.hull(p), want), p.tolist()


def test_matches_brute_force_n64(rng):
    for t in range(6):
        p = workloads.lattice(rng, 64, [1, 3, 7, 100, 1000, 4][t])
        assert same(oracle.hull(p), brute.hull_faces(p))


def test_lower_upper_split_matches_brute_force(rng):
    for p in _degenerate_cases(rng, 120):
        I = np.arange(len(p))
        lo, up = brute.split_lower_upper(p, I, brute.hull_faces(p))
        assert same(oracle.hull(p, lower_only=True), lo)
        assert same(oracle.hull(p, upper_only=True), up)


def test_topdown_equals_bottomup(rng):
    for n in (5, 100, 777, 2048, 3000):
        p = workloads.lattice(rng, n, 30) if n % 2 else workloads.cube(rng, n, 1000)
        assert same(oracle.hull(p), oracle.hull(p, topdown=True))


def test_matches_giftwrap(rng):
    for n, k in ((150, 5), (300, 2000), (512, 100)):
        p = workloads.lattice(rng, n, k)
        assert same(oracle.hull(p), giftwrap.hull_faces(p))


def test_matches_qhull_general_position(rng):
    from scipy.spatial import ConvexHull
    for n in (50, 500, 4096):
        p = workloads.cube(rng, n)
        h = ConvexHull(p.astype(np.float64))
        mine = oracle.hull(p)
        a = {tuple(sorted(f)) for f in mine.tolist()}
        b = {tuple(sorted(f)) for f in h.simplices.tolist()}
        assert a == b
        assert validate.containment_violations(p, mine) == 0


def test_small_n():
    assert oracle.hull(np.zeros((0, 3), np.int32)).shape == (0, 3)
    assert oracle.hull(np.array([[1, 2, 3]])).shape == (0, 3)
    assert oracle.hull(np.array([[1, 2, 3], [4, 5, 6]])).shape == (0, 3)
    f = oracle.hull(np.array([[0, 0, 0], [5, 0, 1], [0, 7, 2]]))
    assert same(f, [[0, 1, 2], [0, 2, 1]])


def test_closed_forms():
    tet = np.array([[0, 0, 0], [10, 0, 0], [0, 10, 0], [0, 0, 10]])
    f = oracle.hull(tet)
    assert len(f) == 4 and validate.containment_violations(tet, f) == 0
    oc = workloads.octahedron(9)
    f = oracle.hull(oc)
    assert len(f) == 8 and validate.euler_ok(f) and validate.manifold_ok(f)
    assert validate.containment_violations(oc, f) == 0
    cu = workloads.cube_corners(4)
    f = oracle.hull(cu)
    assert len(f) == 12 and validate.manifold_ok(f)
    assert validate.containment_violations(cu, f) == 0


def test_cyclic_polytope_gale_evenness():
    """Points on the moment curve, vertex j = j-th value of t: the facets are
    {1, i, i+1} and {i, i+1, N} (Gale's evenness condition in 3-d)."""
    p = workloads.moment_curve(-100, 100)
    N = len(p)
    f = oracle.hull(p)
    want = {(0, i, i + 1) for i in range(1, N - 1)} | {(i, i + 1, N - 1) for i in range(0, N - 2)}
    assert {tuple(sorted(q)) for q in f.tolist()} == want
    assert validate.containment_violations(p, f) == 0
    # shuffled input order: same facets after relabelling
    rng = np.random.default_rng(5)
    perm = rng.permutation(N)
    g = oracle.hull(p[perm])
    assert {tuple(sorted(perm[q])) for q in g.tolist()} == want


@pytest.mark.parametrize("maker", ["cfg1", "ball", "sphere", "gauss"])
def test_invariants_medium(maker):
    rng = np.random.default_rng(11)
    if maker == "cfg1":
        p = workloads.cfg1()
    elif maker == "ball":
        p = workloads.ball(rng, 20000, 1 << 12)
    elif maker == "sphere":
        p = workloads.sphere(rng, 6000, 1 << 12)
    else:
        p = workloads.gaussian(rng, 30000, sigma=1 << 6, clip=1 << 9)
    f = oracle.hull(p)
    assert validate.euler_ok(f)
    assert validate.manifold_ok(f)
    assert len(f) <= 2 * len(p)
    sample = np.random.default_rng(0).choice(len(p), size=min(len(p), 3000), replace=False)
    assert validate.containment_violations(p, f, points=sample) == 0


def test_movies_match_sorted_lower_faces(rng):
    """A block's movie is its lower (or, run 1, upper) faces sorted by event
    time, each the event of its middle vertex; insertion iff D < 0."""
    for t in range(40):
        n = int(rng.integers(4, 40))
        p = workloads.lattice(rng, n, [1, 2, 3, 7, 50][t % 5])
        if t % 6 == 0:
            p[:, 0] = 1
        order = brute.rank_order(p, np.arange(n))
        Ps, Is = p[order], np.arange(n)[order]
        for run in (0, 1):
            for level in range(1, oracle.levels_for(n) + 1):
                ev, bl = oracle.level_movies(p, run, level)
                w = 1 << level
                pos = 0
                for b, s in enumerate(range(0, n, w)):
                    want = brute.block_movie(Ps, Is, np.arange(s, min(s + w, n)), run)
                    got = ev[pos: pos + bl[b]]
                    pos += bl[b]
                    assert got.shape == want.shape and (got == want).all(), (run, level, s)


def test_movie_sizes_and_events(rng):
    p = workloads.cube(rng, 3000, 1 << 20)
    f, st = oracle.hull(p, stats=True)
    for run in (0, 1):
        for level in range(1, oracle.levels_for(len(p)) + 1):
            ev, bl = oracle.level_movies(p, run, level)
            w = 1 << level
            sizes = np.array([min(w, len(p) - s) for s in range(0, len(p), w)])
            assert (bl <= np.maximum(2 * sizes - 5, 0)).all()
            # every point has at most one insertion and one deletion per block
            key = ev[:, 1].astype(np.int64) * 2 + ev[:, 3]
            assert len(np.unique(key)) == len(key)
            merged = np.array([s + w // 2 < min(s + w, len(p)) for s in range(0, len(p), w)])
            assert st[run, level - 1, 1] == bl[merged].sum()
            assert st[run, level - 1, 3] == merged.sum()


def _lower_chain_2d(P, I, ranks):
    """Andrew's monotone chain on the perturbed xy-projection of a block."""
    chain = []
    for r in ranks:
        while len(chain) >= 2 and brute.d_sign(P, I, chain[-2], chain[-1], r) < 0:
            chain.pop()
        chain.append(r)
    return chain


def test_minus_infinity_chains(rng):
    for t in range(30):
        n = int(rng.integers(3, 200))
        p = workloads.lattice(rng, n, [1, 3, 9, 1000][t % 4])
        order = brute.rank_order(p, np.arange(n))
        Ps, Is = p[order], np.arange(n)[order]
        for level in range(1, oracle.levels_for(n) + 1):
            pv, nx = oracle.level_chains(p, t % 2, level)
            w = 1 << level
            for s in range(0, n, w):
                want = _lower_chain_2d(Ps, Is, range(s, min(s + w, n)))
                got = [s]
                while nx[got[-1]] >= 0:
                    got.append(int(nx[got[-1]]))
                assert got == want


def test_rejects_bad_input():
    with pytest.raises(oracle.OracleError) as e:
        oracle.hull(np.array([[0, 0, 1 << 29 + 1], [1, 1, 1], [2, 2, 2]]))
    assert e.value.code == -3

"""Pins for the oracle's symbolic predicates.

The oracle expands D, N and the event-time comparison in epsilon and takes the
first nonzero coefficient.  Here the same quantities are evaluated on points
actually moved by concrete tiny epsilons, in exact big-integer arithmetic
(oracle.perturb): a wrong term, sign, index power or monomial order in the
oracle shows up as a sign mismatch on some of these small, mostly degenerate
inputs.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import brute, perturb


def _rows(P, I):
    return np.concatenate([np.asarray(P, np.int64), np.asarray(I, np.int64)[:, None]], axis=1)


def _tiny_cases(rng, count, coord=2, max_index=15, k=3):
    for _ in range(count):
        P = rng.integers(-coord, coord + 1, size=(k, 3))
        I = rng.choice(max_index + 1, size=k, replace=False)
        yield P, I


def test_D_sign_matches_concrete_epsilon(rng):
    for P, I in _tiny_cases(rng, 3000):
        K = perturb.choose_k(2, 15)
        pz = perturb.Perturbed(P, I, K)
        want = perturb.sign(pz.D(0, 1, 2))
        assert want != 0
        assert oracle.predicate(_rows(P, I), 0) == want


def test_N_sign_matches_concrete_epsilon(rng):
    for P, I in _tiny_cases(rng, 3000):
        K = perturb.choose_k(2, 15)
        pz = perturb.Perturbed(P, I, K)
        assert oracle.predicate(_rows(P, I), 1) == perturb.sign(pz.N(0, 1, 2))


@pytest.mark.parametrize("zsign,which", [(1, 2), (-1, 3)])
def test_time_order_matches_concrete_epsilon(rng, zsign, which):
    """sign(tau_A - tau_B) for pairs of triples, sharing 0..2 points."""
    n_share = 0
    for t in range(4000):
        coord = 2 if t % 2 else 1
        P = rng.integers(-coord, coord + 1, size=(6, 3))
        I = rng.choice(12, size=6, replace=False)
        share = t % 3
        # make the second triple reuse `share` points of the first
        for s in range(share):
            P[3 + s] = P[s]
            I[3 + s] = I[s]
        if len(set(I[:3])) < 3 or len(set(I[3:])) < 3:
            continue
        n_share += share > 0
        K = perturb.choose_k(coord, 12)
        pz = perturb.Perturbed(P, I, K, zsign=zsign)
        want = perturb.sign(pz.tau(0, 1, 2) - pz.tau(3, 4, 5))
        assert oracle.predicate(_rows(P, I), which) == want, (P.tolist(), I.tolist())
    assert n_share > 1000


def test_event_time_symmetric_under_permutation(rng):
    """tau(a, b, c) = N / D is the y-slope of the plane through the three
    points, so it does not depend on their order."""
    for P, I in _tiny_cases(rng, 500, coord=3):
        for perm in itertools.permutations(range(3)):
            rows = np.concatenate([_rows(P, I), _rows(P[list(perm)], I[list(perm)])])
            assert oracle.predicate(rows, 2) == 0
            assert oracle.predicate(rows, 3) == 0


def test_D_never_zero_exhaustive_small():
    """Distinct indices make the perturbed D nonzero, even for coincident
    points: checked on every triple of points from {0,1}^2 x {0}."""
    pts = [(x, y, 0) for x in (0, 1) for y in (0, 1)]
    for trip in itertools.product(pts, repeat=3):
        for I in ((0, 1, 2), (2, 0, 1), (5, 3, 4)):
            rows = _rows(np.array(trip), np.array(I))
            assert oracle.predicate(rows, 0) != 0


def test_brute_orient3d_matches_concrete_epsilon(rng):
    """The numpy epsilon expansion used by brute force and gift-wrap."""
    for t in range(400):
        n = 6
        P = rng.integers(-2, 3, size=(n, 3))
        I = rng.choice(20, size=n, replace=False)
        K = perturb.choose_k(2, 20)
        pz = perturb.Perturbed(P, I, K)
        A, B, C = np.array([0]), np.array([1]), np.array([2])
        sg = brute.orient3d_signs(P, I, A, B, C)[0]
        for d in range(3, n):
            assert sg[d] == perturb.sign(pz.orient3d(0, 1, 2, d))
            assert sg[d] != 0
        assert brute.d_sign(P, I, 0, 1, 2) == perturb.sign(pz.D(0, 1, 2))

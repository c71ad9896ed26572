"""Pins of the oracle's per-level counters (events read, events written,
points touched, merges), which define the algorithmic bytes of every merge
level in the benchmark (CPU only).

Two independent checks:
  * events in / out and merges against the movies themselves
    (``oracle.level_movies`` at levels k - 1 and k);
  * all four counters against a second merge written in plain Python with
    exact rational event times (``oracle.kinetic_py``).
"""
import numpy as np
import pytest

import oracle
from oracle import kinetic_py
from paper_1205_1171_amd import workloads


def _inputs(rng):
    cases = []
    for t in range(24):
        n = int(rng.integers(3, 90))
        p = workloads.lattice(rng, n, [1, 2, 3, 7, 50, 1000][t % 6])
        if t % 5 == 0:
            p[:, 0] = 3            # one x value: the planar blocks of low levels
        if t % 7 == 0:
            p[n // 2:, :] = p[: n - n // 2, :]  # duplicates
        cases.append(p)
    cases.append(workloads.cube(rng, 200, 1 << 20))
    cases.append(workloads.cube(rng, 129, 1 << 10))
    return cases


def test_counters_match_python_recount(rng):
    for p in _inputs(rng):
        _, st = oracle.hull(p, stats=True)
        for run in (0, 1):
            want, _ = kinetic_py.level_counts(p, run)
            L = oracle.levels_for(len(p))
            got = st[run, :L]
            assert (got == want[:L]).all(), (len(p), run, got.tolist(), want[:L].tolist())


def test_events_in_are_child_movie_lengths(rng):
    for p in _inputs(rng)[:12] + [workloads.cube(rng, 3000, 1 << 20)]:
        n = len(p)
        _, st = oracle.hull(p, stats=True)
        for run in (0, 1):
            prev_len = np.zeros(n, dtype=np.int64)   # level 0: every block empty
            for k in range(1, oracle.levels_for(n) + 1):
                w, half = 1 << k, 1 << (k - 1)
                _, bl = oracle.level_movies(p, run, k)
                e_in = e_out = merges = 0
                for b, s in enumerate(range(0, n, w)):
                    if s + half >= min(s + w, n):
                        continue
                    e_in += prev_len[s // half] + prev_len[s // half + 1]
                    e_out += bl[b]
                    merges += 1
                assert st[run, k - 1, 0] == e_in, (n, run, k)
                assert st[run, k - 1, 1] == e_out, (n, run, k)
                assert st[run, k - 1, 3] == merges, (n, run, k)
                prev_len = bl.astype(np.int64)


def test_touched_bounds_and_level_one(rng):
    p = workloads.cube(rng, 1000, 1 << 20)
    _, st = oracle.hull(p, stats=True)
    n = len(p)
    for run in (0, 1):
        # level 1: every merge of two single points splices their links
        assert st[run, 0, 2] == 2 * st[run, 0, 3] == n
        for k in range(1, oracle.levels_for(n) + 1):
            w, half = 1 << k, 1 << (k - 1)
            in_merges = sum(min(s + w, n) - s for s in range(0, n, w) if s + half < min(s + w, n))
            assert 0 < st[run, k - 1, 2] <= in_merges


@pytest.mark.parametrize("run", [0, 1])
def test_python_recount_movie_is_the_oracles(rng, run):
    """The recount's final movie has the oracle's events (same points, same
    order), so the two merges walk the same event sequence."""
    for p in _inputs(rng)[:10]:
        _, mov = kinetic_py.level_counts(p, run)
        ev, _ = oracle.level_movies(p, run, -1)
        assert list(ev[:, 1]) == list(mov)

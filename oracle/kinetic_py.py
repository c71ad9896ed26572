"""A second sequential kinetic merge, in plain Python, that recounts the
oracle's per-level counters (test infrastructure).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.  It shares nothing
with ``minimalist.c`` but the method: the bottom-up level loop over blocks of
2^k ranks (Sec. 2, the movie array; Sec. 3, Fig. "main_loop_figure"), Chan's
merge of two movies (the bridge at t = -inf, the six candidate events, the
rewind to the merged -inf chain), and the act() toggle (Fig.
"act_functions").  Predicates are not expanded in epsilon: every point is
moved by concrete tiny epsilons and scaled to integers (``perturb``), so a
triple's event time tau = N / D is an exact ``Fraction`` and events compare
as (tau, rank triple) tuples.

Counters per run and level (the algorithmic-bytes model of the benchmark):
  events_in      child-movie events of the level's merges,
  events_out     events of the merged movies,
  points_touched distinct points whose coordinates a merge of the level reads
                 (a predicate) or whose links it changes (act, the -inf splice,
                 the rewind),
  merges         pairs of blocks merged.
Small inputs only (a few hundred points): every predicate is a big-integer
determinant.
"""
from fractions import Fraction

import numpy as np

from . import perturb

NIL = -1


class _Run:
    def __init__(self, P, I, zsign):
        K = perturb.choose_k(int(np.abs(P).max(initial=1)), int(np.max(I, initial=1)))
        self.pp = perturb.Perturbed(P, I, K, zsign)
        n = len(P)
        self.prev = [NIL] * n
        self.next = [NIL] * n
        self.seen = set()

    def touch(self, *ps):
        for p in ps:
            if p != NIL:
                self.seen.add(p)

    def d_sign(self, a, b, c):
        self.touch(a, b, c)
        return perturb.sign(self.pp.D(a, b, c))

    def event(self, l, m, r):
        """(time, key) of the triple l < m < r: orders events strictly."""
        self.touch(l, m, r)
        return (Fraction(self.pp.N(l, m, r), self.pp.D(l, m, r)), (l, m, r))

    def toggle(self, p):
        """Insert p between its stored neighbours, or unlink it if the left
        neighbour already points at it."""
        pv, nx = self.prev[p], self.next[p]
        self.touch(p, pv, nx)
        if self.next[pv] != p:
            self.next[pv] = p
            self.prev[nx] = p
        else:
            self.next[pv] = nx
            self.prev[nx] = pv


def _merge(R, m, Lmov, Rmov):
    prev, nxt = R.prev, R.next
    u, v = m - 1, m
    # lower common tangent of the two xy chains at t = -inf
    while True:
        if nxt[v] != NIL and R.d_sign(u, v, nxt[v]) < 0:
            v = nxt[v]
        elif prev[u] != NIL and R.d_sign(prev[u], u, v) < 0:
            u = prev[u]
        else:
            break
    i = j = 0
    out = []
    last = None
    while True:
        cands = []
        if i < len(Lmov):
            w = Lmov[i]
            cands.append((R.event(prev[w], w, nxt[w]), 0))
        if j < len(Rmov):
            w = Rmov[j]
            cands.append((R.event(prev[w], w, nxt[w]), 1))
        if nxt[u] != NIL:
            cands.append((R.event(u, nxt[u], v), 2))
        if prev[u] != NIL:
            cands.append((R.event(prev[u], u, v), 3))
        if prev[v] != NIL:
            cands.append((R.event(u, prev[v], v), 4))
        if nxt[v] != NIL:
            cands.append((R.event(u, v, nxt[v]), 5))
        later = [c for c in cands if last is None or c[0] > last]
        if not later:
            break
        ev, slot = min(later)
        last = ev
        if slot == 0:
            w = Lmov[i]
            i += 1
            if w < u:
                out.append(w)
            R.toggle(w)
        elif slot == 1:
            w = Rmov[j]
            j += 1
            if w > v:
                out.append(w)
            R.toggle(w)
        elif slot == 2:
            u = nxt[u]
            out.append(u)
        elif slot == 3:
            out.append(u)
            u = prev[u]
        elif slot == 4:
            v = prev[v]
            out.append(v)
        else:
            out.append(v)
            v = nxt[v]
    # back to t = -inf: the merged chain, and every point off it pointing at
    # the neighbours it will be inserted between
    R.touch(u, v)
    nxt[u] = v
    prev[v] = u
    for w in reversed(out):
        if w <= u or w >= v:
            R.toggle(w)
            if w == u:
                u = prev[u]
            elif w == v:
                v = nxt[v]
        else:
            R.touch(w, u, v)
            nxt[u] = w
            prev[w] = u
            prev[v] = w
            nxt[w] = v
            if w < m:
                u = w
            else:
                v = w
    return out


def level_counts(xyz, run):
    """Counters of the bottom-up driver on one run (0 lower, 1 upper):
    int64 [L, 4] = (events_in, events_out, points_touched, merges) per level,
    and the final movie (point ranks)."""
    P = np.asarray(xyz, dtype=np.int64).reshape(-1, 3)
    n = len(P)
    I = np.arange(n)
    order = np.lexsort((I, P[:, 0]))
    R = _Run(P[order], I[order], 1 if run == 0 else -1)
    L = 0
    while (1 << L) < n:
        L += 1
    movies = {s: [] for s in range(n)}
    stats = np.zeros((max(L, 1), 4), dtype=np.int64)
    for k in range(1, L + 1):
        w, half = 1 << k, 1 << (k - 1)
        R.seen = set()
        nxt = {}
        for s in range(0, n, w):
            m = s + half
            if m >= min(s + w, n):
                nxt[s] = movies[s]
                continue
            stats[k - 1, 0] += len(movies[s]) + len(movies[m])
            nxt[s] = _merge(R, m, movies[s], movies[m])
            stats[k - 1, 1] += len(nxt[s])
            stats[k - 1, 3] += 1
        stats[k - 1, 2] = len(R.seen)
        movies = nxt
    return stats, movies.get(0, [])

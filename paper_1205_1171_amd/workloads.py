"""Seeded synthetic point clouds (int32 xyz, C-contiguous [n, 3]).

This module only draws inputs; it holds none of the hull's arithmetic, and
both the GPU path and the CPU oracle consume what it produces.  The paper
states no point distribution for its runtime table (Sec. 4), so the workloads
below are the project's own, sized like the paper's largest runs:

  cfg1          n = 4096 uniform in [-2^20, 2^20]^3, x values distinct
  cfg2-sphere   n = 2^20 on the sphere of radius 2^20 (lattice-rounded)
  cfg2-ball     n = 2^20 lattice-uniform in the ball of radius 2^20
  cfg3          n = 2^24: 99% Gaussian (sigma 2^16, clipped to +-2^20) and
                1% on the sphere of radius 2^20, rows shuffled
  cfg4          10,000 clouds, sizes floor(2^U), U ~ U[3, 16], each a ball or
                a sphere of radius 2^20 with probability 1/2
  cfg5          256 clouds of 16,384 points near the sphere of radius 2^18
                (radial Gaussian noise, sigma 2^10): float32 positions and the
                int32 lattice points they round to

Exact duplicate rows are redrawn in every workload.
"""
import numpy as np

SEED = 12051171
R20 = 1 << 20


def rng_for(cfg, sub=0):
    """Generator for workload ``cfg`` (1..5); ``sub`` separates sub-workloads."""
    if sub == 0:
        return np.random.Generator(np.random.PCG64(SEED + cfg))
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED + cfg, sub])))


def _row_keys(p):
    q = p.astype(np.int64) + R20 * 4
    base = np.uint64(R20 * 8 + 1)
    return (q[:, 0].astype(np.uint64) * base + q[:, 1].astype(np.uint64)) * base + q[:, 2].astype(np.uint64)


def later_duplicates(p):
    """Row positions that repeat an earlier row exactly."""
    if len(p) == 0:
        return np.zeros(0, dtype=np.int64)
    if np.abs(p).max() > R20 * 4:
        raise ValueError("coordinates outside the generator's key range")
    key = _row_keys(p)
    _, first = np.unique(key, return_index=True)
    dup = np.ones(len(p), dtype=bool)
    dup[first] = False
    return np.nonzero(dup)[0]


def _redraw(p, draw, rng, groups=None):
    """Redraw every later duplicate with ``draw(rng, k[, group])`` until none."""
    for _ in range(1000):
        d = later_duplicates(p)
        if len(d) == 0:
            return p
        if groups is None:
            p[d] = draw(rng, len(d))
        else:
            for g in np.unique(groups[d]):
                sel = d[groups[d] == g]
                p[sel] = draw(rng, len(sel), g)
    raise RuntimeError("could not remove duplicates")


def sphere(rng, n, radius=R20):
    g = rng.standard_normal((n, 3))
    nrm = np.linalg.norm(g, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return np.rint(radius * g / nrm).astype(np.int32)


def ball(rng, n, radius=R20):
    out = np.empty((0, 3), dtype=np.int32)
    r2 = radius * radius
    while len(out) < n:
        k = int((n - len(out)) * 2.0) + 16
        c = rng.integers(-radius, radius, size=(k, 3), endpoint=True, dtype=np.int64)
        keep = (c * c).sum(axis=1) <= r2
        out = np.concatenate([out, c[keep].astype(np.int32)])
    return out[:n]


def cube(rng, n, half=R20):
    return rng.integers(-half, half, size=(n, 3), endpoint=True, dtype=np.int64).astype(np.int32)


def gaussian(rng, n, sigma=1 << 16, clip=R20):
    g = np.rint(rng.normal(0.0, sigma, size=(n, 3)))
    return np.clip(g, -clip, clip).astype(np.int32)


def cfg1(n=4096):
    rng = rng_for(1)
    p = cube(rng, n)
    for _ in range(1000):
        _, first = np.unique(p[:, 0], return_index=True)
        rep = np.ones(n, dtype=bool)
        rep[first] = False
        d = np.nonzero(rep)[0]
        if len(d) == 0:
            break
        p[d] = cube(rng, len(d))
    return np.ascontiguousarray(p)


def cfg2_sphere(n=1 << 20):
    rng = rng_for(2)
    p = sphere(rng, n)
    return np.ascontiguousarray(_redraw(p, lambda r, k: sphere(r, k), rng))


def cfg2_ball(n=1 << 20):
    rng = rng_for(2, sub=1)
    p = ball(rng, n)
    return np.ascontiguousarray(_redraw(p, lambda r, k: ball(r, k), rng))


def cfg3(n=1 << 24, sphere_frac=0.01):
    rng = rng_for(3)
    ns = int(round(sphere_frac * n))
    ng = n - ns
    p = np.concatenate([sphere(rng, ns), gaussian(rng, ng)])
    comp = np.concatenate([np.zeros(ns, np.int8), np.ones(ng, np.int8)])
    perm = rng.permutation(n)
    p, comp = p[perm], comp[perm]

    def draw(r, k, g):
        return sphere(r, k) if g == 0 else gaussian(r, k)

    return np.ascontiguousarray(_redraw(p, draw, rng, comp))


def cfg4(H=10000, lo=3.0, hi=16.0):
    """Concatenated clouds and int64 offsets [H + 1]."""
    rng = rng_for(4)
    sizes = np.floor(2.0 ** rng.uniform(lo, hi, size=H)).astype(np.int64)
    kinds = rng.integers(0, 2, size=H)
    parts = []
    for s, k in zip(sizes, kinds):
        if k == 0:
            q = _redraw(ball(rng, int(s)), lambda r, m: ball(r, m), rng)
        else:
            q = _redraw(sphere(rng, int(s)), lambda r, m: sphere(r, m), rng)
        parts.append(q)
    off = np.zeros(H + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return np.ascontiguousarray(np.concatenate(parts)), off, kinds


def noisy_sphere(rng, m, radius=float(1 << 18), sigma=float(1 << 10)):
    g = rng.standard_normal((m, 3))
    nrm = np.linalg.norm(g, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    r = radius + rng.normal(0.0, sigma, size=(m, 1))
    return (g / nrm * r).astype(np.float32)


def cfg5(B=256, m=16384):
    """float32 positions [B, m, 3] and their int32 lattice points [B, m, 3]."""
    rng = rng_for(5)
    P = np.empty((B, m, 3), dtype=np.float32)
    for b in range(B):
        p = noisy_sphere(rng, m)
        for _ in range(1000):
            q = np.rint(p).astype(np.int32)
            d = later_duplicates(q)
            if len(d) == 0:
                break
            p[d] = noisy_sphere(rng, len(d))
        P[b] = p
    return P, np.rint(P).astype(np.int32)


def lattice(rng, n, k):
    """n points with coordinates in {0..k}^3 (heavy ties, duplicates kept)."""
    return rng.integers(0, k, size=(n, 3), endpoint=True, dtype=np.int64).astype(np.int32)


def octahedron(k):
    return np.array([[k, 0, 0], [-k, 0, 0], [0, k, 0], [0, -k, 0], [0, 0, k], [0, 0, -k]],
                    dtype=np.int32)


def cube_corners(k):
    return np.array([[x, y, z] for x in (0, k) for y in (0, k) for z in (0, k)], dtype=np.int32)


def moment_curve(t0=-100, t1=100):
    """Points (t, t^2, t^3): every one a vertex of their hull (cyclic polytope)."""
    t = np.arange(t0, t1 + 1, dtype=np.int64)
    return np.stack([t, t * t, t * t * t], axis=1).astype(np.int32)


def planar(n=1 << 18):
    """Delaunay workload: n distinct int32 points uniform in [-2^14, 2^14]^2
    (the lifting range), [n, 2]."""
    rng = rng_for(6)
    draw = lambda r, k: r.integers(-(1 << 14), 1 << 14, size=(k, 2), endpoint=True)
    p = draw(rng, n)
    for _ in range(1000):
        key = (p[:, 0] + (1 << 15)) * (1 << 16) + (p[:, 1] + (1 << 15))
        _, first = np.unique(key, return_index=True)
        dup = np.ones(n, dtype=bool)
        dup[first] = False
        d = np.nonzero(dup)[0]
        if len(d) == 0:
            break
        p[d] = draw(rng, len(d))
    return np.ascontiguousarray(p.astype(np.int32))


def planar_wide(n=1 << 18):
    """Delaunay workload on the full lifting range: n distinct int32 points
    uniform in [-2^20, 2^20]^2 (lifted z up to 2^41), [n, 2]."""
    rng = rng_for(7)
    draw = lambda r, k: r.integers(-R20, R20, size=(k, 2), endpoint=True)
    p = draw(rng, n)
    for _ in range(1000):
        key = (p[:, 0] + 2 * R20) * (4 * R20 + 1) + (p[:, 1] + 2 * R20)
        _, first = np.unique(key, return_index=True)
        dup = np.ones(n, dtype=bool)
        dup[first] = False
        d = np.nonzero(dup)[0]
        if len(d) == 0:
            break
        p[d] = draw(rng, len(d))
    return np.ascontiguousarray(p.astype(np.int32))


def float_ball(n=1 << 20):
    """Float-input workload: n float32 points uniform in the unit ball
    (rejection from the cube, in float64, then rounded to float32), [n, 3].
    On the 30-bit lattice (scale 2^30, as the largest |c| is just below 1)
    every coordinate of magnitude at least 2^-7 keeps its float32 value
    exactly."""
    rng = rng_for(8)
    out = np.empty((0, 3))
    while len(out) < n:
        c = rng.uniform(-1.0, 1.0, size=(2 * n, 3))
        out = np.concatenate([out, c[(c * c).sum(axis=1) <= 1.0]])
    return np.ascontiguousarray(out[:n].astype(np.float32))

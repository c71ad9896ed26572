"""The oracle: a plain, sequential, exact CPU implementation of the kinetic
3-d convex hull (Sec. 2 "Algorithm" and Sec. 3 "Implementation" of the paper),
plus the independent checks that pin it.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.
It shares no code with the GPU library and imports nothing from it.

Modules
-------
``minimalist.c``  the sequential minimalist hull (C, exact 256-bit arithmetic),
                  loaded here through ctypes.
``perturb``       perturbed predicates evaluated at concrete tiny epsilons with
                  exact big integers (the pin for the symbolic perturbation).
``brute``         O(n^4) brute-force hull and block movies (plain definition).
``giftwrap``      an independent gift-wrapping hull under the same perturbation.
``validate``      canonical form, Euler count, closed-manifold and containment.
``volume_area``   FP64 hull volume and area and their gradients.
``adjacency``     face adjacency (half-edge twins) of a face list.
``delaunay``      2-d Delaunay by lifting, and the in-circle pin.
``floatin``       float input: the snap to an integer lattice with a
                  power-of-two scale, then the exact hull (wide range).
``kinetic_py``    a second merge in Python that recounts the level counters.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "minimalist.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build():
    """Compile the C oracle (gcc, host only)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _SO)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    lib.oracle_sort.argtypes = [P, i64, P]
    lib.oracle_hull.argtypes = [P, i64, i32, P, i64, P, P, i32]
    lib.oracle_level_movies.argtypes = [P, i64, i32, i32, P, i64, P, P]
    lib.oracle_level_chains.argtypes = [P, i64, i32, i32, P, P]
    lib.oracle_predicate.argtypes = [P, i32, i32]
    lib.oracle_hull_wide.argtypes = [P, i64, i32, P, i64, P]
    for f in (lib.oracle_sort, lib.oracle_hull, lib.oracle_level_movies,
              lib.oracle_level_chains, lib.oracle_predicate, lib.oracle_hull_wide):
        f.restype = i32
    _lib = lib
    return lib


def _pts(xyz):
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.int32).reshape(-1, 3))
    return a, a.shape[0]


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle returned status {code}")
        self.code = code


def sort_order(xyz):
    """Input index of the point of each rank (order by x, then input index)."""
    a, n = _pts(xyz)
    out = np.empty(n, dtype=np.int32)
    rc = _load().oracle_sort(a.ctypes.data, n, out.ctypes.data)
    if rc:
        raise OracleError(rc)
    return out


def levels_for(n):
    L = 0
    while (1 << L) < n:
        L += 1
    return L


def hull(xyz, lower_only=False, upper_only=False, topdown=False, stats=False):
    """Outward face triples (input indices): lower run's faces, then upper's.

    With ``stats`` (bottom-up only) also returns an int64 array [2, L, 4]:
    per run and level, (events read, events written, points touched, merges).
    """
    a, n = _pts(xyz)
    flags = (1 if lower_only else 0) | (2 if topdown else 0) | (4 if upper_only else 0)
    cap = max(2 * n, 1)
    faces = np.empty((cap, 3), dtype=np.int32)
    nf = ctypes.c_int64(0)
    L = max(levels_for(n), 1)
    st = np.zeros((2, L, 4), dtype=np.int64)
    rc = _load().oracle_hull(a.ctypes.data, n, flags, faces.ctypes.data, cap,
                             ctypes.addressof(nf), st.ctypes.data if stats else None, L)
    if rc:
        raise OracleError(rc)
    f = faces[: nf.value].copy()
    return (f, st) if stats else f


def hull_wide(xyz, lower_only=False, upper_only=False, topdown=False):
    """hull() on int64 rows over the wide range |x|, |y| <= 2^30, |z| <= 2^42
    (the same method, predicates and perturbation)."""
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.int64).reshape(-1, 3))
    n = a.shape[0]
    flags = (1 if lower_only else 0) | (2 if topdown else 0) | (4 if upper_only else 0)
    cap = max(2 * n, 1)
    faces = np.empty((cap, 3), dtype=np.int32)
    nf = ctypes.c_int64(0)
    rc = _load().oracle_hull_wide(a.ctypes.data, n, flags, faces.ctypes.data, cap,
                                  ctypes.addressof(nf))
    if rc:
        raise OracleError(rc)
    return faces[: nf.value].copy()


def level_movies(xyz, run, level):
    """Movies after ``level`` bottom-up levels of run 0 (lower) / 1 (upper).

    Returns (events [E,4] = left, middle, right rank and is_insertion,
    per-block lengths) with blocks of width 2^level from rank 0.
    """
    a, n = _pts(xyz)
    cap = max(2 * n, 1)
    ev = np.empty((cap, 4), dtype=np.int32)
    width = 1 << min(level if level >= 0 else levels_for(n), levels_for(max(n, 1)))
    nb = max((n + width - 1) // width, 1)
    bl = np.zeros(nb, dtype=np.int64)
    tot = ctypes.c_int64(0)
    rc = _load().oracle_level_movies(a.ctypes.data, n, run, level, ev.ctypes.data, cap,
                                     bl.ctypes.data, ctypes.addressof(tot))
    if rc:
        raise OracleError(rc)
    return ev[: tot.value].copy(), bl


def level_chains(xyz, run, level):
    """(prev, next) by rank of every block's -inf chain after ``level`` levels."""
    a, n = _pts(xyz)
    pv = np.empty(n, dtype=np.int32)
    nx = np.empty(n, dtype=np.int32)
    rc = _load().oracle_level_chains(a.ctypes.data, n, run, level, pv.ctypes.data, nx.ctypes.data)
    if rc:
        raise OracleError(rc)
    return pv, nx


def predicate(rows, which):
    """Exact perturbed predicate on rows (x, y, z, index): see minimalist.c."""
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1, 4))
    return int(_load().oracle_predicate(r.ctypes.data, r.shape[0], which))

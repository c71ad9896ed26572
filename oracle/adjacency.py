"""Face adjacency (half-edge twins) of a triangulated surface: the plain
definition, test infrastructure only.

Face row f = (v0, v1, v2) has the directed edges k = 0: v0 -> v1,
k = 1: v1 -> v2, k = 2: v2 -> v0.  Its neighbour across edge k is the face
holding the reverse directed edge (v_{k+1} -> v_k); on a closed, consistently
oriented surface that face exists and is unique.  adj[f, k] is its row, -1
when no face holds the reverse edge.

In a batch, clouds are separate surfaces: an edge matches only within its own
cloud (its vertices are indices within the cloud).
"""
import numpy as np


def adjacency(faces, face_off=None):
    """adj [F, 3] int32 by a dictionary of directed edges (the definition)."""
    f = np.asarray(faces, dtype=np.int64).reshape(-1, 3)
    F = len(f)
    off = np.array([0, F], dtype=np.int64) if face_off is None else np.asarray(face_off, np.int64)
    adj = np.full((F, 3), -1, dtype=np.int32)
    for h in range(len(off) - 1):
        owner = {}
        for r in range(off[h], off[h + 1]):
            for k in range(3):
                owner[(int(f[r, k]), int(f[r, (k + 1) % 3]))] = r
        for r in range(off[h], off[h + 1]):
            for k in range(3):
                adj[r, k] = owner.get((int(f[r, (k + 1) % 3]), int(f[r, k])), -1)
    return adj


def adjacency_sorted(faces, face_off=None, pt_off=None):
    """The same map for large face sets (vectorised: sorted directed-edge
    keys, then a search for each reversed key).  Vertices are made global
    with the clouds' point offsets (pt_off) when given, else keyed by
    (cloud, vertex), which needs fewer than 2^9 clouds."""
    f = np.asarray(faces, dtype=np.int64).reshape(-1, 3)
    F = len(f)
    off = np.array([0, F], dtype=np.int64) if face_off is None else np.asarray(face_off, np.int64)
    cloud = np.repeat(np.arange(len(off) - 1, dtype=np.int64), np.diff(off))
    a = f
    b = np.roll(f, -1, axis=1)
    if pt_off is not None:
        base = np.asarray(pt_off, np.int64)[cloud][:, None]
        ga, gb = a + base, b + base
        assert ga.max(initial=0) < (1 << 31)
        key, rkey = (ga << 31) | gb, (gb << 31) | ga
    else:
        assert len(off) - 1 < (1 << 9) and f.max(initial=0) < (1 << 27)
        key = (cloud[:, None] << 54) | (a << 27) | b
        rkey = (cloud[:, None] << 54) | (b << 27) | a
    kf = key.ravel()
    order = np.argsort(kf, kind="stable")
    ks = kf[order]
    pos = np.searchsorted(ks, rkey.ravel())
    pos = np.minimum(pos, len(ks) - 1)
    hit = ks[pos] == rkey.ravel()
    twin_half = np.where(hit, order[pos], -1)
    adj = np.where(twin_half >= 0, twin_half // 3, -1).astype(np.int32)
    return adj.reshape(F, 3)

"""Writes the stored expected values for the full-size parity tests.

Calls only the oracle (``oracle/``) and the seeded input generators: for each
workload it records the oracle's face count, vertex count, the SHA-256 of its
canonical face array (oracle.validate.canonical, int32 little-endian) for the
full hull and for the lower hull, and the oracle's per-level counters of the
bottom-up driver (events read, events written, points touched, merges) that
define the algorithmic bytes of each merge level.

For the batched workload cfg4 (10,000 clouds of 8 to 65,536 points) it
records, per cloud in cloud order, the oracle's face count, and the SHA-256
of the concatenation of every cloud's canonical face array (indices local to
the cloud).

For the Delaunay workloads (planar: 2^18 points in [-2^14, 2^14]^2;
planar_wide: 2^18 points in [-2^20, 2^20]^2) it records the SHA-256 of the
oracle's canonical triangle array; for the float-input workload (float_ball:
2^20 float32 points in the unit ball, on the 30-bit lattice) the face count
and the SHA-256 of the oracle's canonical faces (full and lower).

For the differentiation workload cfg5 (256 clouds of 16,384 float32 points,
hulls on their int32 lattice points) it records, per cloud, the oracle's face
count, the SHA-256 of the concatenated canonical face arrays, the FP64 volume
and area of each cloud (float64 positions of the float32 points, the oracle's
faces), and the FP64 gradient of a seeded weighted loss sum_b wV[b] V_b +
wA[b] A_b at 16 seeded vertices of every cloud.

usage: python tests/golden/make_golden.py cfg1 cfg2_sphere cfg2_ball cfg3 cfg4 cfg5 planar
       planar_wide float_ball
(the lower and upper runs go to two processes; the clouds of cfg4 to a pool)
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle import validate  # noqa: E402
from paper_1205_1171_amd import workloads  # noqa: E402

MAKERS = {
    "cfg1": workloads.cfg1,
    "cfg2_sphere": workloads.cfg2_sphere,
    "cfg2_ball": workloads.cfg2_ball,
    "cfg3": workloads.cfg3,
}


def digest(faces):
    c = validate.canonical(faces).astype("<i4")
    return hashlib.sha256(c.tobytes()).hexdigest()


def _run(args):
    name, which = args
    p = MAKERS[name]()
    t = time.time()
    f, st = oracle.hull(p, lower_only=which == 0, upper_only=which == 1, stats=True)
    return which, f, st[which], time.time() - t


def _cloud(q):
    t = time.time()
    return validate.canonical(oracle.hull(q)).astype("<i4"), time.time() - t


def make_batched(name, workers):
    pts, off, kinds = workloads.cfg4()
    clouds = [pts[off[h]:off[h + 1]] for h in range(len(off) - 1)]
    order = np.argsort([-len(c) for c in clouds], kind="stable")  # longest first
    res = [None] * len(clouds)
    t = time.time()
    with ProcessPoolExecutor(workers) as ex:
        for h, r in zip(order, ex.map(_cloud, [clouds[h] for h in order], chunksize=4)):
            res[h] = r
    sha = hashlib.sha256()
    for f, _ in res:
        sha.update(f.tobytes())
    rec = {
        "config": name,
        "H": int(len(clouds)),
        "n": int(off[-1]),
        "input_sha256": hashlib.sha256(np.ascontiguousarray(pts, dtype="<i4").tobytes()).hexdigest(),
        "offsets_sha256": hashlib.sha256(off.astype("<i8").tobytes()).hexdigest(),
        "F": int(sum(len(f) for f, _ in res)),
        "F_per_cloud": [int(len(f)) for f, _ in res],
        "sha256_full": sha.hexdigest(),
        "oracle_seconds_cpu": float(sum(s for _, s in res)),
        "oracle_seconds_wall": time.time() - t,
        "oracle_workers": workers,
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(rec, fh)
    print(name, rec["F"], rec["oracle_seconds_cpu"], rec["oracle_seconds_wall"], flush=True)


CFG5_GRAD_SEED = 12051175
CFG5_GRAD_VERTS = 16


def _cloud5(args):
    from oracle import volume_area as va
    P32, Pi, b, wV, wA, seed = args
    t = time.time()
    f = oracle.hull(Pi)
    P64 = P32.astype(np.float64)
    V, A = va.volume_area(P64, f)
    gV, gA = va.gradients(P64, f)
    rng = np.random.default_rng([seed, b])
    verts = rng.choice(np.unique(f), CFG5_GRAD_VERTS, replace=False)
    g = wV * gV[verts] + wA * gA[verts]
    return validate.canonical(f).astype("<i4"), V, A, verts, g, time.time() - t


def make_cfg5(name, workers):
    P, Pi = workloads.cfg5()
    B = len(P)
    wrng = np.random.default_rng(CFG5_GRAD_SEED)
    wV = wrng.standard_normal(B)
    wA = wrng.standard_normal(B)
    t = time.time()
    jobs = [(P[b], Pi[b], b, float(wV[b]), float(wA[b]), CFG5_GRAD_SEED) for b in range(B)]
    with ProcessPoolExecutor(workers) as ex:
        res = list(ex.map(_cloud5, jobs, chunksize=2))
    sha = hashlib.sha256()
    for r in res:
        sha.update(r[0].tobytes())
    rec = {
        "config": name,
        "B": int(B),
        "m": int(P.shape[1]),
        "input_sha256": hashlib.sha256(np.ascontiguousarray(Pi, dtype="<i4").tobytes()).hexdigest(),
        "positions_sha256": hashlib.sha256(np.ascontiguousarray(P, dtype="<f4").tobytes()).hexdigest(),
        "F": int(sum(len(r[0]) for r in res)),
        "F_per_cloud": [int(len(r[0])) for r in res],
        "sha256_full": sha.hexdigest(),
        "V64": [float(r[1]) for r in res],
        "A64": [float(r[2]) for r in res],
        "grad_seed": CFG5_GRAD_SEED,
        "grad_wV": [float(x) for x in wV],
        "grad_wA": [float(x) for x in wA],
        "grad_vertices": [[int(v) for v in r[3]] for r in res],
        "grad64": [[[float(x) for x in row] for row in r[4]] for r in res],
        "oracle_seconds_cpu": float(sum(r[5] for r in res)),
        "oracle_seconds_wall": time.time() - t,
        "oracle_workers": workers,
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(rec, fh)
    print(name, rec["F"], rec["oracle_seconds_cpu"], rec["oracle_seconds_wall"], flush=True)


def make_delaunay(name):
    """A Delaunay workload: the oracle's lifted lower hull, CCW triangles."""
    from oracle import delaunay as dl
    p = workloads.planar() if name == "planar" else workloads.planar_wide()
    t = time.time()
    tris = dl.delaunay(p)
    rec = {
        "config": name,
        "n": int(len(p)),
        "input_sha256": hashlib.sha256(np.ascontiguousarray(p, dtype="<i4").tobytes()).hexdigest(),
        "T": int(len(tris)),
        "sha256": digest(tris),
        "oracle_seconds": time.time() - t,
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(name, rec["T"], rec["oracle_seconds"], flush=True)


def make_float(name, bits=30):
    """The float-input workload: the oracle's hull of the float32 points
    snapped to the 30-bit lattice (lower and upper runs)."""
    from oracle import floatin
    p = workloads.float_ball()
    t = time.time()
    lower = floatin.hull_f32(p, bits, lower_only=True)
    faces = floatin.hull_f32(p, bits)
    rec = {
        "config": name,
        "n": int(len(p)),
        "bits": bits,
        "input_sha256": hashlib.sha256(np.ascontiguousarray(p, dtype="<f4").tobytes()).hexdigest(),
        "F": int(len(faces)),
        "F_lower": int(len(lower)),
        "V": int(validate.vertex_count(faces)),
        "euler_ok": bool(validate.euler_ok(faces)),
        "sha256_full": digest(faces),
        "sha256_lower": digest(lower),
        "oracle_seconds": time.time() - t,
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(name, rec["F"], rec["V"], rec["oracle_seconds"], flush=True)


def make(name):
    if name in ("planar", "planar_wide"):
        return make_delaunay(name)
    if name == "float_ball":
        return make_float(name)
    if name == "cfg4":
        return make_batched(name, int(os.environ.get("GOLDEN_WORKERS", "6")))
    if name == "cfg5":
        return make_cfg5(name, int(os.environ.get("GOLDEN_WORKERS", "6")))
    p = MAKERS[name]()
    with ProcessPoolExecutor(2) as ex:
        res = sorted(ex.map(_run, [(name, 0), (name, 1)]), key=lambda r: r[0])
    lower, upper = res[0][1], res[1][1]
    faces = np.concatenate([lower, upper])
    rec = {
        "config": name,
        "n": int(len(p)),
        "input_sha256": hashlib.sha256(np.ascontiguousarray(p, dtype="<i4").tobytes()).hexdigest(),
        "F": int(len(faces)),
        "F_lower": int(len(lower)),
        "V": int(validate.vertex_count(faces)),
        "euler_ok": bool(validate.euler_ok(faces)),
        "manifold_ok": bool(validate.manifold_ok(faces)),
        "sha256_full": digest(faces),
        "sha256_lower": digest(lower),
        "level_stats_columns": ["events_in", "events_out", "points_touched", "merges"],
        "level_stats_lower": res[0][2].tolist(),
        "level_stats_upper": res[1][2].tolist(),
        "oracle_seconds_lower": res[0][3],
        "oracle_seconds_upper": res[1][3],
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(name, rec["F"], rec["V"], rec["oracle_seconds_lower"], rec["oracle_seconds_upper"],
          flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:]:
        make(name)

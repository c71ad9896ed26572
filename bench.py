"""Throughput of the MI355X kinetic 3-d hull.

One step = one hull_full call (range check, radix sort by x, every merge
level of the lower and upper runs, face extraction) on the n = 2^24 workload
(99% Gaussian, 1% sphere), inputs resident in HBM.  Prints one JSON line:
value = Mpoints/s = n / (time per step).

Also reported:
  roofline      the merge-level kernel: algorithmic bytes per launch (from the
                oracle's per-level counters: 4 B per event read, 4 B per
                event written, 28 B per point touched) over its average launch
                time, measured with HIP events recorded around every merge
                launch on the library's stream during the timed steps;
  cpu_baseline  the oracle (sequential C, one thread) on a bounded sample of
                the same workload.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg3]
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _hip():
    for name in ("libamdhip64.so", "libamdhip64.so.7", "/opt/rocm/lib/libamdhip64.so"):
        try:
            return ctypes.CDLL(name)
        except OSError:
            continue
    raise RuntimeError("libamdhip64 not found")


class Events:
    """A block of hipEvent_t handles created through the HIP runtime."""

    def __init__(self, count):
        self.hip = _hip()
        self.arr = (ctypes.c_void_p * count)()
        for q in range(count):
            rc = self.hip.hipEventCreate(ctypes.byref(self.arr, q * ctypes.sizeof(ctypes.c_void_p)))
            if rc:
                raise RuntimeError(f"hipEventCreate failed: {rc}")

    def ms(self, a, b):
        out = ctypes.c_float(0)
        rc = self.hip.hipEventElapsedTime(ctypes.byref(out), ctypes.c_void_p(self.arr[a]),
                                          ctypes.c_void_p(self.arr[b]))
        if rc:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return out.value

    def close(self):
        for q in range(len(self.arr)):
            self.hip.hipEventDestroy(ctypes.c_void_p(self.arr[q]))


def levels_for(n):
    L = 0
    while (1 << L) < n:
        L += 1
    return L


def cpu_baseline(p, sample_n):
    """The oracle, as it stands, on the first sample_n rows (rows are in
    random order, so this is a uniform subsample of the same workload)."""
    import oracle
    s = p[:sample_n].copy()
    t = time.perf_counter()
    f = oracle.hull(s)
    dt = time.perf_counter() - t
    return {"value": round(sample_n / dt / 1e6, 6), "unit": "Mpoints/s", "cores": 1,
            "kind": "oracle",
            "sample": f"first {sample_n} rows of the workload (uniform subsample), lower+upper "
                      f"runs, sequential C oracle, {dt:.1f} s, {len(f)} faces"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--cpu-sample", type=int, default=1 << 17)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the hull is not "
              "distributed across GPUs.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1205_1171_amd import hull, workloads
    L_ = hull.lib()
    maker = {"cfg1": workloads.cfg1, "cfg2_sphere": workloads.cfg2_sphere,
             "cfg2_ball": workloads.cfg2_ball, "cfg3": workloads.cfg3}[args.workload]
    p = maker()
    n = len(p)
    print(f"[bench] workload {args.workload} n={n}", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(p).to(dev)
    cap = 2 * n
    faces = torch.empty((cap, 3), dtype=torch.int32, device=dev)
    info = torch.zeros(2, dtype=torch.int64, device=dev)
    ws = torch.empty(hull.workspace_bytes(n), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    sptr = ctypes.c_void_p(stream.cuda_stream)
    L = levels_for(n)
    nev = 2 * L + 3
    ev = Events(nev * max(args.steps, 1))

    def step(k=None):
        if k is None:
            rc = L_.hull_full(ctypes.c_void_p(x.data_ptr()), n, ctypes.c_void_p(faces.data_ptr()),
                              cap, ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), sptr)
        else:
            arr = ctypes.cast(ctypes.byref(ev.arr, k * nev * ctypes.sizeof(ctypes.c_void_p)),
                              ctypes.c_void_p)
            rc = L_.hull_full_timed(ctypes.c_void_p(x.data_ptr()), n,
                                    ctypes.c_void_p(faces.data_ptr()), cap,
                                    ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                    ws.numel(), sptr, arr, nev)
        if rc:
            raise hull.HullError(rc, "hull_full")

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)
    st, F = (int(v) for v in info.cpu())
    if st:
        raise hull.HullError(st, "device")

    # bit-exactness of the last warmup result against the oracle's digest
    bit_exact = None
    gpath = os.path.join(ROOT, "tests", "golden", f"{args.workload}.json")
    golden = json.load(open(gpath)) if os.path.exists(gpath) else None
    if golden is not None:
        from oracle import validate
        g = faces[:F].cpu().numpy()
        bit_exact = (len(g) == golden["F"] and hashlib.sha256(
            validate.canonical(g).astype("<i4").tobytes()).hexdigest() == golden["sha256_full"])

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[bench] timed {args.steps} steps", file=sys.stderr, flush=True)
    ms = (t1 - t0) * 1000.0 / args.steps

    # per-level merge kernel times (ms), averaged over the timed steps
    lvl = np.zeros(L)
    sort_ms = extract_ms = 0.0
    for k in range(args.steps):
        b = k * nev
        sort_ms += ev.ms(b + 0, b + 1)
        extract_ms += ev.ms(b + 2 * L + 1, b + 2 * L + 2)
        for q in range(1, L + 1):
            lvl[q - 1] += ev.ms(b + 2 * q, b + 2 * q + 1)
    lvl /= args.steps
    sort_ms /= args.steps
    extract_ms /= args.steps
    ev.close()

    roofline = None
    if golden is not None:
        stats = np.array(golden["level_stats_lower"]) + np.array(golden["level_stats_upper"])
        Bk = 4 * stats[:, 0] + 4 * stats[:, 1] + 28 * stats[:, 2]   # bytes per level
        per_launch = float(Bk.sum()) / L
        avg_s = float(lvl.mean()) / 1000.0
        achieved = per_launch / avg_s / 1e9
        traffic = None
        tpath = os.path.join(ROOT, "profiles", f"merge_level_{args.workload}_traffic.json")
        if os.path.exists(tpath):
            tr = json.load(open(tpath))
            src = open(os.path.join(ROOT, "paper_1205_1171_amd", "csrc", "merge.hip"), "rb").read()
            if tr.get("merge_source_sha256") == hashlib.sha256(src).hexdigest():
                traffic = tr.get("bytes_per_launch")
        roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
                    "kernel": "k_merge_level", "launches_per_step": L,
                    "avg_launch_ms": round(float(lvl.mean()), 4),
                    "algorithmic_bytes_per_launch": per_launch}

    out = {
        "metric": "Mpoints/s per hull (n=2^24)",
        "value": round(n / (ms / 1000.0) / 1e6, 4),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: n={n}", "n": n, "faces": F,
                   "runs": "lower+upper"},
        "bit_exact": bit_exact,
        "phase_ms": {"sort": round(sort_ms, 4), "merge_levels": [round(v, 4) for v in lvl],
                     "extract": round(extract_ms, 4)},
        "roofline": roofline,
    }
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(p, min(args.cpu_sample, n))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

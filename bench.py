"""Throughput of the MI355X kinetic 3-d hull.

One step = one hull_full call (range check, radix sort by x, every merge
level of the lower and upper runs, face extraction) on the n = 2^24 workload
(99% Gaussian, 1% sphere), inputs resident in HBM.  Prints one JSON line:
value = Mpoints/s = n / (time per step).

Also reported on the same line:
  roofline        the merge kernel with the largest share of the step (the
                  lane-serial k_merge_level_lk with its links in LDS, or
                  k_merge_level, the lane-group k_merge_wave or the
                  LDS-staged k_merge_level_lds, whichever takes the most
                  time over its levels): algorithmic bytes per launch (from
                  the oracle's per-level counters: 4 B per event read, 4 B
                  per event written, 28 B per point touched) over its average
                  launch time, measured with HIP events recorded around each
                  of its launches on the library's stream in the timed steps,
                  and the HBM traffic per launch that rocprofv3's FETCH_SIZE
                  and WRITE_SIZE counters read for it (profiles/, while the
                  merge sources are the ones profiled);
  levels          the same figure for every merge level (the parallel levels
                  are several kernels each, timed as a whole);
  other_single_hulls  Mpoints/s and bit-exact flags on n = 4096 and the
                  n = 2^20 sphere and ball;
  delaunay        2-d Delaunay by lifting (lower hull of (x, y, x^2 + y^2)) on
                  2^18 points, Mpoints/s and bit-exact flag;
  batched         10,000 ragged clouds (7.3e7 points) in one hull_full_batched
                  call captured in a HIP graph, against one hull_full launch
                  per cloud on the same stream (hulls/s), schedule from the
                  autotuner's cache;
  differentiation 256 clouds x 16,384 points: FP32 volume/area forward +
                  backward for all clouds in one launch each, against one
                  launch per cloud, with and without the batched hull first;
  adjacency       face adjacency (half-edge twins) of the n = 2^24 hull's faces
                  and of the 10,000-cloud batch's faces;
  cpu_baseline    the oracle (sequential C, one thread) on a bounded sample of
                  the n = 2^24 workload, with the host's CPU model and core
                  count; and the oracle on every 64th cloud of the batch on a
                  thread pool over the host cores (hulls/s).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg3]
                       [--no-singles] [--no-batched] [--no-diff] [--no-per-hull]
                       [--no-cpu]
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


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


def timed(fn, reps):
    """Average ms of fn() over reps calls, timed with events on torch's
    current stream (where the library launches)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def host_cpu():
    """CPU model and the number of cores this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, len(os.sched_getaffinity(0)), os.cpu_count()


def cpu_baseline(p, sample_n):
    """The oracle, as it stands, on the first sample_n rows (rows are in
    random order, so this is a uniform subsample of the same workload).  The
    method is sequential: one thread."""
    import oracle
    s = p[:sample_n].copy()
    t = time.perf_counter()
    f = oracle.hull(s)
    dt = time.perf_counter() - t
    model, avail, total = host_cpu()
    return {"value": round(sample_n / dt / 1e6, 6), "unit": "Mpoints/s", "cores": 1,
            "kind": "oracle", "cpu_model": model, "nproc": avail, "cpu_count": total,
            "sample": f"first {sample_n} rows of the n = 2^24 workload (a uniform subsample), "
                      f"lower+upper runs, sequential C oracle on one thread, {dt:.1f} s, "
                      f"{len(f)} faces"}


def cpu_batched(workloads, stride=64, max_threads=16):
    """The oracle on every stride-th cloud of the 10,000-cloud batch (the same
    size and kind mix), one cloud per task on a thread pool over the host
    cores this process may use (at most max_threads: the GPU machine's share);
    the C oracle runs outside the Python lock.  Hulls/s and Mpoints/s."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    pts, off, _ = workloads.cfg4()
    idx = list(range(0, len(off) - 1, stride))
    clouds = [np.ascontiguousarray(pts[off[h]:off[h + 1]]) for h in idx]
    clouds.sort(key=len, reverse=True)  # longest first
    model, avail, total = host_cpu()
    threads = max(1, min(avail, max_threads))
    t = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        faces = sum(len(f) for f in ex.map(oracle.hull, clouds))
    dt = time.perf_counter() - t
    npts = sum(len(c) for c in clouds)
    return {"hulls_per_s": round(len(clouds) / dt, 2), "Mpoints_per_s": round(npts / dt / 1e6, 4),
            "cores": threads, "kind": "oracle", "cpu_model": model, "nproc": avail,
            "sample": f"every {stride}th cloud of the 10,000-cloud batch ({len(clouds)} clouds, "
                      f"{npts} points, {faces} faces), thread pool of {threads}, {dt:.1f} s"}


def single(args, hull, workloads):
    import numpy as np
    import torch
    L_ = hull.lib()
    maker = {"cfg1": workloads.cfg1, "cfg2_sphere": workloads.cfg2_sphere,
             "cfg2_ball": workloads.cfg2_ball, "cfg3": workloads.cfg3}[args.workload]
    p = maker()
    n = len(p)
    log(f"workload {args.workload} n={n}")
    dev = torch.device("cuda:0")
    x = torch.from_numpy(p).to(dev)
    cap = 2 * n
    faces = torch.empty((cap, 3), dtype=torch.int32, device=dev)
    info = torch.zeros(2, dtype=torch.int64, device=dev)
    ws = torch.empty(hull.workspace_bytes(n), dtype=torch.uint8, device=dev)
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = levels_for(n)
    nev = 2 * L + 3
    ev = Events(nev * max(args.steps, 1))
    sched = hull.schedule_defaults()

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
        log(f"warmup {w} done")
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
    log(f"timed {args.steps} steps")
    ms = (t1 - t0) * 1000.0 / args.steps

    # per-level merge times (ms), averaged over the timed steps
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

    adj_ms = adjacency_ms(hull, faces[:F])
    roofline = levels = None
    S = min(sched.serial_levels, L)
    KL = min(sched.fused_levels, S)  # lowest levels: the LDS-staged kernel
    W = sched.wave_from if sched.wave_from > 0 else L + 1  # first lane-group level
    lds_links = os.environ.get("HULL_LDS_LINKS", "1") != "0"

    def kernel_of(k):  # k: 1-based level
        if k > S:
            return "parallel strategy (k_par_* kernels, device scans)"
        if k <= KL:
            return "k_merge_level_lds"
        if k >= W:
            return "k_merge_wave"
        # lane-serial blocks of up to 128 points keep their links in LDS
        return "k_merge_level_lk" if lds_links and k <= 7 else "k_merge_level"

    if golden is not None:
        stats = np.array(golden["level_stats_lower"]) + np.array(golden["level_stats_upper"])
        Bk = 4.0 * stats[:, 0] + 4.0 * stats[:, 1] + 28.0 * stats[:, 2]  # bytes per level
        levels = [{"level": k + 1, "kernel": kernel_of(k + 1),
                   "ms": round(float(lvl[k]), 4), "algorithmic_bytes": float(Bk[k]),
                   "GBps": round(float(Bk[k]) / (lvl[k] / 1e3) / 1e9, 2),
                   "frac": round(float(Bk[k]) / (lvl[k] / 1e3) / 1e9 / HBM_PEAK_GBS, 6)}
                  for k in range(L)]
        # the dominant kernel: the merge kernel with the most time in the step
        groups = {}
        for k in range(L):
            kn = kernel_of(k + 1)
            if not kn.startswith("parallel"):
                groups.setdefault(kn, []).append(k)
        if groups:
            kern, ks = max(groups.items(), key=lambda t: float(lvl[t[1]].sum()))
            per_launch = float(Bk[ks].sum()) / len(ks)
            avg_ms = float(lvl[ks].mean())
            achieved = per_launch / (avg_ms / 1e3) / 1e9
            traffic = None
            tpath = os.path.join(ROOT, "profiles", f"{kern}_{args.workload}_traffic.json")
            if os.path.exists(tpath):
                tr = json.load(open(tpath))
                src = b"".join(open(os.path.join(ROOT, "paper_1205_1171_amd", "csrc", f), "rb").read()
                               for f in ("merge.hip", "merge_wave.hpp", "events.hpp",
                                         "predicates.hpp"))
                if (tr.get("source_sha256") == hashlib.sha256(src).hexdigest()
                        and tr.get("levels") == [ks[0] + 1, ks[-1] + 1]):
                    traffic = tr.get("hbm_bytes_per_launch")
            roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6),
                        "traffic": traffic, "kernel": kern,
                        "levels": [ks[0] + 1, ks[-1] + 1], "launches_per_step": len(ks),
                        "avg_launch_ms": round(avg_ms, 4),
                        "algorithmic_bytes_per_launch": per_launch,
                        "all_levels_GBps": round(float(Bk.sum()) / (lvl.sum() / 1e3) / 1e9, 3)}

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
        "config": {"workload": f"{args.workload}: n={n} (99% Gaussian sigma 2^16 clipped to "
                               f"+-2^20, 1% sphere radius 2^20)" if args.workload == "cfg3"
                   else f"{args.workload}: n={n}",
                   "n": n, "faces": F, "runs": "lower+upper",
                   "schedule": {"serial_levels": sched.serial_levels,
                                "walk_segment": sched.walk_segment,
                                "wave_from": sched.wave_from,
                                "wave_lanes": sched.wave_lanes,
                                "wave_lanes_max": sched.wave_lanes_max}},
        "bit_exact": bit_exact,
        "phase_ms": {"sort": round(sort_ms, 4), "merge_levels": [round(v, 4) for v in lvl],
                     "extract": round(extract_ms, 4)},
        # sort: range pass 12 B/pt, 3 radix passes of 16 B/pt (key + index read
        # and written), gather 12 B/pt read + 16 B/pt written (22-bit keys)
        "sort": {"ms": round(sort_ms, 4), "algorithmic_bytes": 88.0 * n,
                 "GBps": round(88.0 * n / (sort_ms / 1e3) / 1e9, 1)},
        "roofline": roofline,
        "levels": levels,
        "adjacency": {"faces": F, "ms": round(adj_ms, 4),
                      "Mfaces_per_s": round(F / (adj_ms / 1e3) / 1e6, 1)},
    }
    return out, p


def adjacency_ms(hull, faces, face_off=None, pt_off=None, reps=5):
    """Average ms of hull_face_adjacency on a face set (workspace and output
    allocated once, outside the timed calls)."""
    import torch
    L_ = hull.lib()
    F = faces.shape[0]
    faces = faces.contiguous()
    adj = torch.empty((max(F, 1), 3), dtype=torch.int32, device="cuda")
    info = torch.empty(2, dtype=torch.int64, device="cuda")
    nb = ctypes.c_size_t(0)
    L_.hull_adjacency_workspace_bytes(F, ctypes.byref(nb))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    H = 1 if face_off is None else face_off.numel() - 1
    P = ctypes.c_void_p

    def call():
        rc = L_.hull_face_adjacency(P(faces.data_ptr()), F,
                                    P(face_off.data_ptr()) if face_off is not None else None,
                                    P(pt_off.data_ptr()) if pt_off is not None else None, H,
                                    P(adj.data_ptr()), P(info.data_ptr()), P(ws.data_ptr()),
                                    ws.numel(), sptr)
        if rc:
            raise hull.HullError(rc, "hull_face_adjacency")

    call()
    ms = timed(call, reps)
    st, open_edges = (int(v) for v in info.cpu())
    if st or open_edges:
        raise RuntimeError(f"adjacency: status {st}, {open_edges} open edges")
    return ms


def other_singles(hull, workloads, reps=5):
    """Mpoints/s of hull_full on the other single-hull workloads, each
    checked against the oracle's digest."""
    import torch
    from oracle import validate
    L_ = hull.lib()
    out = {}
    for name in ("cfg1", "cfg2_sphere", "cfg2_ball"):
        p = getattr(workloads, name)()
        n = len(p)
        x = torch.from_numpy(p).cuda()
        faces = torch.empty((2 * n, 3), dtype=torch.int32, device="cuda")
        info = torch.zeros(2, dtype=torch.int64, device="cuda")
        ws = torch.empty(hull.workspace_bytes(n), dtype=torch.uint8, device="cuda")
        sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

        def call():
            rc = L_.hull_full(ctypes.c_void_p(x.data_ptr()), n, ctypes.c_void_p(faces.data_ptr()),
                              2 * n, ctypes.c_void_p(info.data_ptr()),
                              ctypes.c_void_p(ws.data_ptr()), ws.numel(), sptr)
            if rc:
                raise hull.HullError(rc, "hull_full")

        call()
        call()
        st, F = (int(v) for v in info.cpu())
        g = json.load(open(os.path.join(ROOT, "tests", "golden", f"{name}.json")))
        exact = (st == 0 and F == g["F"] and hashlib.sha256(validate.canonical(
            faces[:F].cpu().numpy()).astype("<i4").tobytes()).hexdigest() == g["sha256_full"])
        ms = timed(call, reps)
        # the same hull through the batched entry point (one cloud) captured
        # in a HIP graph: no per-kernel launch cost
        bh = hull.BatchedHull(x, [0, n])
        bh.capture()
        bh.replay()
        ms_g = timed(bh.replay, reps)
        fg, _ = bh.result()
        same = fg.shape[0] == F and hashlib.sha256(validate.canonical(
            fg.cpu().numpy()).astype("<i4").tobytes()).hexdigest() == g["sha256_full"]
        out[name] = {"n": n, "faces": F, "ms": round(ms, 4),
                     "Mpoints_per_s": round(n / (ms / 1e3) / 1e6, 2), "bit_exact": exact,
                     "ms_graph": round(ms_g, 4),
                     "Mpoints_per_s_graph": round(n / (ms_g / 1e3) / 1e6, 2),
                     "bit_exact_graph": same}
        del bh
        log(f"{name}: {out[name]}")
        del x, faces, ws
    return out


def delaunay_line(hull, workloads, reps=5):
    """Delaunay by lifting on 2^18 points of [-2^14, 2^14]^2: Mpoints/s and
    the bit-exact flag against the oracle's digest."""
    import torch
    from oracle import validate
    L_ = hull.lib()
    p = workloads.planar()
    n = len(p)
    x = torch.from_numpy(p).cuda()
    tris = torch.empty((2 * n, 3), dtype=torch.int32, device="cuda")
    info = torch.zeros(2, dtype=torch.int64, device="cuda")
    nb = ctypes.c_size_t(0)
    L_.hull_delaunay_workspace_bytes(n, ctypes.byref(nb))
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def call():
        rc = L_.hull_delaunay(ctypes.c_void_p(x.data_ptr()), n, ctypes.c_void_p(tris.data_ptr()),
                              2 * n, ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), sptr)
        if rc:
            raise hull.HullError(rc, "hull_delaunay")

    call()
    st, T = (int(v) for v in info.cpu())
    exact = None
    gpath = os.path.join(ROOT, "tests", "golden", "planar.json")
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        exact = (st == 0 and T == g["T"] and hashlib.sha256(validate.canonical(
            tris[:T].cpu().numpy()).astype("<i4").tobytes()).hexdigest() == g["sha256"])
    ms = timed(call, reps)
    return {"workload": f"planar: {n} distinct points uniform in [-2^14, 2^14]^2", "n": n,
            "triangles": T, "ms": round(ms, 4), "Mpoints_per_s": round(n / (ms / 1e3) / 1e6, 2),
            "bit_exact": exact}


def batched(hull, workloads, autotune, reps, per_hull=True):
    """cfg4: one graph-captured batched call against one call per cloud."""
    import numpy as np
    import torch
    L_ = hull.lib()
    pts, off, _ = workloads.cfg4()
    H = len(off) - 1
    N = int(off[-1])
    log(f"batched workload: {H} clouds, {N} points")
    x = torch.from_numpy(pts).cuda()
    sched = autotune.lookup(off)
    bh = hull.BatchedHull(x, off, sched)
    bh.run()
    faces, face_off = bh.result()
    bit_exact = None
    gpath = os.path.join(ROOT, "tests", "golden", "cfg4.json")
    if os.path.exists(gpath):
        from oracle import validate
        rec = json.load(open(gpath))
        f = faces.cpu().numpy()
        fo = face_off.cpu().numpy()
        sha = hashlib.sha256()
        for h in range(H):
            sha.update(validate.canonical(f[fo[h]:fo[h + 1]]).astype("<i4").tobytes())
        bit_exact = (np.diff(fo).tolist() == rec["F_per_cloud"]
                     and sha.hexdigest() == rec["sha256_full"])
    log(f"batched bit_exact={bit_exact}")
    ms_eager = timed(bh.run, reps)
    bh.capture()
    bh.replay()
    ms_graph = timed(bh.replay, reps)
    log(f"batched graph {ms_graph:.2f} ms, eager {ms_eager:.2f} ms")

    # one hull_full call per cloud, same stream, one workspace for the largest
    sizes = np.diff(off)
    nmax = int(sizes.max())
    ws = torch.empty(hull.workspace_bytes(nmax), dtype=torch.uint8, device="cuda")
    fbuf = torch.empty((2 * nmax, 3), dtype=torch.int32, device="cuda")
    info = torch.zeros(2, dtype=torch.int64, device="cuda")
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    base = x.data_ptr()

    def run_per_hull(count):
        for h in range(count):
            rc = L_.hull_full(ctypes.c_void_p(base + 12 * int(off[h])), int(sizes[h]),
                              ctypes.c_void_p(fbuf.data_ptr()), fbuf.shape[0],
                              ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                              ws.numel(), sptr)
            if rc:
                raise hull.HullError(rc, "hull_full")

    ms_loop = None
    if per_hull:
        run_per_hull(min(H, 200))  # warm-up
        ms_loop = timed(lambda: run_per_hull(H), 1)
        log(f"one launch per cloud: {ms_loop:.1f} ms")
    # face adjacency (half-edge twins) of the batch's faces
    adj_ms = adjacency_ms(hull, faces, face_off, torch.from_numpy(off).cuda())
    s = sched if sched is not None else hull.schedule_defaults()
    return {
        "workload": f"cfg4: {H} clouds, sizes floor(2^U), U ~ U[3,16], 50/50 ball/sphere of "
                    f"radius 2^20, {N} points",
        "hulls": H, "points": N, "faces": int(face_off[-1]),
        "schedule": {"serial_levels": s.serial_levels, "walk_segment": s.walk_segment,
                     "wave_from": s.wave_from, "wave_lanes": s.wave_lanes,
                     "wave_lanes_max": s.wave_lanes_max,
                     "source": "autotuner cache" if sched is not None else "library defaults"},
        "ms_graph": round(ms_graph, 3), "ms_eager": round(ms_eager, 3),
        "ms_one_launch_per_hull": round(ms_loop, 3) if ms_loop else None,
        "hulls_per_s": round(H / (ms_graph / 1e3), 1),
        "hulls_per_s_eager": round(H / (ms_eager / 1e3), 1),
        "hulls_per_s_one_launch_per_hull": round(H / (ms_loop / 1e3), 1) if ms_loop else None,
        "speedup_vs_one_launch_per_hull": round(ms_loop / ms_graph, 2) if ms_loop else None,
        "Mpoints_per_s": round(N / (ms_graph / 1e3) / 1e6, 2),
        "bit_exact": bit_exact,
        "adjacency": {"faces": int(face_off[-1]), "ms": round(adj_ms, 3),
                      "Mfaces_per_s": round(int(face_off[-1]) / (adj_ms / 1e3) / 1e6, 1)},
    }


def differentiation(hull, workloads, autotune, reps):
    """cfg5: FP32 volume/area forward + backward, batched against per cloud."""
    import numpy as np
    import torch
    P, Q = workloads.cfg5()
    B, m = P.shape[0], P.shape[1]
    log(f"differentiation workload: {B} clouds x {m} points")
    p = torch.from_numpy(P.reshape(-1, 3)).cuda()
    x = torch.from_numpy(np.ascontiguousarray(Q.reshape(-1, 3))).cuda()
    off = np.arange(0, B * m + 1, m, dtype=np.int64)
    d_off = torch.from_numpy(off).cuda()
    bh = hull.BatchedHull(x, off, autotune.lookup(off))
    bh.run()
    faces, face_off = bh.result()
    faces = faces.contiguous()
    gV = torch.ones(B, dtype=torch.float32, device="cuda")
    gA = torch.ones(B, dtype=torch.float32, device="cuda")

    def fb_batched():
        hull.volume_area_fwd(p, d_off, faces, face_off)
        hull.volume_area_bwd(p, d_off, faces, face_off, gV, gA)

    fo = face_off.cpu().numpy()
    one_off = torch.tensor([0, m], dtype=torch.int64, device="cuda")
    cloud_face_off = [torch.tensor([0, int(fo[b + 1] - fo[b])], dtype=torch.int64, device="cuda")
                      for b in range(B)]
    L_ = hull.lib()
    Vb = torch.empty(1, dtype=torch.float32, device="cuda")
    Ab = torch.empty(1, dtype=torch.float32, device="cuda")
    g = torch.empty((m, 3), dtype=torch.float32, device="cuda")
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    P_ = ctypes.c_void_p

    def fb_cloud(b):
        pp = P_(p.data_ptr() + 12 * b * m)
        ff = P_(faces.data_ptr() + 12 * int(fo[b]))
        rc = L_.hull_volume_area_fwd(pp, P_(one_off.data_ptr()), ff,
                                     P_(cloud_face_off[b].data_ptr()), 1, P_(Vb.data_ptr()),
                                     P_(Ab.data_ptr()), sptr)
        rc = rc or L_.hull_volume_area_bwd(pp, P_(one_off.data_ptr()), ff,
                                           P_(cloud_face_off[b].data_ptr()), 1,
                                           P_(gV.data_ptr()), P_(gA.data_ptr()),
                                           P_(g.data_ptr()), sptr)
        if rc:
            raise hull.HullError(rc, "volume/area")

    def fb_per_cloud():
        for b in range(B):
            fb_cloud(b)

    ws = torch.empty(hull.workspace_bytes(m), dtype=torch.uint8, device="cuda")
    fbuf = torch.empty((2 * m, 3), dtype=torch.int32, device="cuda")
    info = torch.zeros(2, dtype=torch.int64, device="cuda")

    def hull_fb_per_cloud():
        for b in range(B):
            rc = L_.hull_full(P_(x.data_ptr() + 12 * b * m), m, P_(fbuf.data_ptr()), fbuf.shape[0],
                              P_(info.data_ptr()), P_(ws.data_ptr()), ws.numel(), sptr)
            if rc:
                raise hull.HullError(rc, "hull_full")
            fb_cloud(b)

    def hull_fb_batched():
        bh.run()
        fb_batched()

    fb_batched()
    fb_per_cloud()
    ms_b = timed(fb_batched, reps)
    ms_c = timed(fb_per_cloud, reps)
    hull_fb_per_cloud()
    ms_hb = timed(hull_fb_batched, reps)
    ms_hc = timed(hull_fb_per_cloud, 1)
    V, A = hull.volume_area_fwd(p, d_off, faces, face_off)
    ok = bool(torch.isfinite(V).all() and torch.isfinite(A).all() and (V > 0).all())
    log(f"fwd+bwd batched {ms_b:.3f} ms, per cloud {ms_c:.3f} ms")
    check = diff_check(hull, p, d_off, faces, face_off, V, A, B, m)
    return {
        "workload": f"cfg5: {B} clouds x {m} points on a sphere of radius 2^18 with radial "
                    f"noise sigma 2^10, FP32",
        "clouds": B, "faces": int(fo[-1]),
        "ms_fwd_bwd_batched": round(ms_b, 4), "ms_fwd_bwd_one_launch_per_cloud": round(ms_c, 4),
        "speedup_fwd_bwd": round(ms_c / ms_b, 2),
        "ms_hull_fwd_bwd_batched": round(ms_hb, 3),
        "ms_hull_fwd_bwd_one_launch_per_cloud": round(ms_hc, 3),
        "speedup_with_hull": round(ms_hc / ms_hb, 2),
        "finite_positive_volumes": ok,
        **check,
    }


def diff_check(hull, p, d_off, faces, face_off, V, A, B, m):
    """The differentiation workload's results against the oracle's stored
    values: the canonical face digest of all clouds, V and A of every cloud
    (FP64), and the gradient of the stored weighted loss at the stored
    sampled vertices (FP64)."""
    import numpy as np
    import torch
    from oracle import validate
    gpath = os.path.join(ROOT, "tests", "golden", "cfg5.json")
    if not os.path.exists(gpath):
        return {"bit_exact": None}
    rec = json.load(open(gpath))
    f = faces.cpu().numpy()
    fo = face_off.cpu().numpy()
    sha = hashlib.sha256()
    for b in range(B):
        sha.update(validate.canonical(f[fo[b]:fo[b + 1]]).astype("<i4").tobytes())
    exact = np.diff(fo).tolist() == rec["F_per_cloud"] and sha.hexdigest() == rec["sha256_full"]
    V, A = V.cpu().numpy().astype(np.float64), A.cpu().numpy().astype(np.float64)
    V64, A64 = np.array(rec["V64"]), np.array(rec["A64"])
    wV = torch.tensor(rec["grad_wV"], dtype=torch.float32, device="cuda")
    wA = torch.tensor(rec["grad_wA"], dtype=torch.float32, device="cuda")
    G = hull.volume_area_bwd(p, d_off, faces, face_off, wV, wA)
    G = G.cpu().numpy().reshape(B, m, 3).astype(np.float64)
    gerr = 0.0
    for b in range(B):
        g64 = np.array(rec["grad64"][b])
        g32 = G[b, rec["grad_vertices"][b]]
        gerr = max(gerr, float(np.linalg.norm(g32 - g64) / np.linalg.norm(g64)))
    return {"bit_exact": bool(exact),
            "max_rel_err_V": float(np.max(np.abs(V - V64) / np.abs(V64))),
            "max_rel_err_A": float(np.max(np.abs(A - A64) / np.abs(A64))),
            "max_rel_err_grad": gerr,
            "tolerances": {"V": 1e-5, "A": 1e-5, "grad": 1e-4}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg3")
    ap.add_argument("--cpu-sample", type=int, default=1 << 17)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-diff", action="store_true")
    ap.add_argument("--no-singles", action="store_true",
                    help="skip the n = 4096 and n = 2^20 single-hull lines")
    ap.add_argument("--no-per-hull", action="store_true",
                    help="skip the one-launch-per-cloud comparison (for short profiles)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the hull is not "
              "distributed across GPUs.", file=sys.stderr)
        sys.exit(2)

    from paper_1205_1171_amd import autotune, hull, workloads
    hull.lib()
    out, p = single(args, hull, workloads)
    if not args.no_singles:
        out["other_single_hulls"] = other_singles(hull, workloads)
        out["delaunay"] = delaunay_line(hull, workloads)
    if not args.no_batched:
        out["batched"] = batched(hull, workloads, autotune, reps=3,
                                 per_hull=not args.no_per_hull)
    if not args.no_diff:
        out["differentiation"] = differentiation(hull, workloads, autotune, reps=5)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(p, min(args.cpu_sample, len(p)))
        if not args.no_batched:
            log("cpu batched (oracle, thread pool)")
            out["cpu_baseline"]["batched"] = cpu_batched(workloads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

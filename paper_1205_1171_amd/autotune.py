"""Schedule autotuner for batched hulls (host side).

The merge schedule of hull_full_batched -- how many bottom levels run one
lane per merge, from which of those levels a merge runs on a group of lanes
(and how many at most, as the groups grow by level), and how many child
events each walk segment of the parallel levels takes -- changes nothing in
the result, only the time.  The tuner
times a grid of schedules on the caller's own batch (HIP events on the
current stream, the same kernels the call would run) and keeps the fastest
per device and batch shape in a JSON cache next to this file.  Lookups read
the cache only; a missing entry gives the library defaults.
"""
import json
import math
import os

from . import hull

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned_schedules.json")

SERIAL_LEVELS = (9, 10, 11, 12, 13, 14, 15, 99)
WALK_SEGMENTS = (4, 8, 16, 32)
WAVE_LEVELS = (-1, 5, 6, 7, 8, 9)  # -1: no lane groups
WAVE_LANES = 8
WAVE_LANES_MAX = (8, 64)  # lanes per merge stay at 8, or double per level up to 64


def shape_key(offsets):
    """Batch shape: hull count and the largest and total point counts, each
    rounded to a power of two."""
    import numpy as np
    off = np.asarray(offsets, dtype=np.int64)
    sizes = np.diff(off)
    H = len(sizes)
    mx = int(sizes.max()) if H else 0
    tot = int(off[-1]) if H else 0

    def p2(v):
        return 0 if v <= 1 else int(math.ceil(math.log2(v)))

    return f"H2^{p2(H)}_max2^{p2(mx)}_total2^{p2(tot)}"


def device_key():
    """Architecture and compute-unit count, e.g. gfx950_256CU."""
    import torch
    if not torch.cuda.is_available():
        return "cpu"
    pr = torch.cuda.get_device_properties(0)
    return f"{pr.gcnArchName.split(':')[0]}_{pr.multi_processor_count}CU"


def _load():
    if os.path.exists(CACHE):
        with open(CACHE) as fh:
            return json.load(fh)
    return {}


def lookup(offsets):
    """The cached schedule for this batch shape on this device, or None."""
    rec = _load().get(device_key(), {}).get(shape_key(offsets))
    if rec is None:
        return None
    return hull.Schedule(rec["serial_levels"], rec["walk_segment"], 0, rec.get("wave_from", -1),
                         rec.get("wave_lanes", WAVE_LANES), rec.get("wave_lanes_max", 0))


def tune(xyz, offsets, reps=2, serial_levels=SERIAL_LEVELS, walk_segments=WALK_SEGMENTS,
         wave_levels=WAVE_LEVELS, wave_lanes=WAVE_LANES, wave_lanes_max=WAVE_LANES_MAX, save=True,
         log=None):
    """Time every schedule of the grid on this batch; returns (best Schedule,
    {(serial_levels, walk_segment, wave_from, wave_lanes_max): ms}).  Without
    lane groups (wave_from -1) the lane cap plays no part and is timed once."""
    import torch
    times = {}
    bh = hull.BatchedHull(xyz, offsets)
    base_F = None
    for sl in serial_levels:
        for wf in wave_levels:
            if wf > 0 and wf > sl:
                continue  # no lane-serial level left for the lane groups
            for cap in (wave_lanes_max if wf > 0 else wave_lanes_max[-1:]):
                for seg in walk_segments:
                    bh.schedule = hull.Schedule(sl, seg, 0, wf, wave_lanes, cap)
                    bh.run()
                    torch.cuda.synchronize()
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    for _ in range(reps):
                        bh.run()
                    e1.record()
                    torch.cuda.synchronize()
                    ms = e0.elapsed_time(e1) / reps
                    st, F = (int(v) for v in bh.info.cpu())
                    if st:
                        raise hull.HullError(st, "device")
                    if base_F is None:
                        base_F = F
                    elif F != base_F:
                        raise RuntimeError(f"schedule ({sl}, {seg}, {wf}, {cap}) changed the face count")
                    times[(sl, seg, wf, cap)] = ms
                    if log:
                        log(f"[tune] serial_levels={sl} walk_segment={seg} wave_from={wf} "
                            f"wave_lanes_max={cap}: {ms:.3f} ms")
    (sl, seg, wf, cap), ms = min(times.items(), key=lambda kv: kv[1])
    if save:
        cache = _load()
        cache.setdefault(device_key(), {})[shape_key(offsets)] = {
            "serial_levels": sl, "walk_segment": seg, "wave_from": wf, "wave_lanes": wave_lanes,
            "wave_lanes_max": cap, "ms": round(ms, 4), "reps": reps,
            "grid": {f"{a}:{b}:{c}:{d}": round(v, 4) for (a, b, c, d), v in sorted(times.items())}}
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return hull.Schedule(sl, seg, 0, wf, wave_lanes, cap), times

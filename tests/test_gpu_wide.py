"""GPU parity of the wide coordinate range (int64 rows, |x|, |y| <= 2^30,
|z| <= 2^42) and of float input snapped to a lattice, through the C ABI,
against the oracle's wide entry (oracle.hull_wide) and its float snap
(oracle.floatin).  Bit-exact canonical face sets, under every merge
strategy; full-size float workload against the oracle's stored digest."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from oracle import floatin, validate
from paper_1205_1171_amd import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
XY, Z = 1 << 30, 1 << 42

STRATEGIES = {
    "serial": {"HULL_SERIAL_LEVELS": "99", "HULL_WALK_SEGMENT": "", "HULL_WAVE_LEVEL": "-1"},
    "parallel_seg4": {"HULL_SERIAL_LEVELS": "0", "HULL_WALK_SEGMENT": "4", "HULL_WAVE_LEVEL": "-1"},
    "wave5": {"HULL_SERIAL_LEVELS": "99", "HULL_WALK_SEGMENT": "", "HULL_WAVE_LEVEL": "5"},
    "default": {"HULL_SERIAL_LEVELS": "", "HULL_WALK_SEGMENT": "", "HULL_WAVE_LEVEL": ""},
}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def H():
    import torch
    from paper_1205_1171_amd import hull
    assert torch.cuda.is_available()
    hull.lib()
    return hull


@pytest.fixture(scope="module")
def ws(H):
    return H.Workspace()


@pytest.fixture(params=sorted(STRATEGIES))
def strategy(request):
    saved = {k: os.environ.get(k) for k in STRATEGIES[request.param]}
    os.environ.update(STRATEGIES[request.param])
    yield request.param
    for k, v in saved.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


def same(a, b):
    a, b = validate.canonical(a), validate.canonical(b)
    return a.shape == b.shape and bool((a == b).all())


def wide_faces(H, ws, p, lower_only=False):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(p, dtype=np.int64)).cuda()
    return H.hull_wide(x, lower_only=lower_only, ws=ws).cpu().numpy()


def f32_faces(H, ws, p, bits, lower_only=False):
    import torch
    x = torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()
    return H.hull_f32(x, bits, lower_only=lower_only, ws=ws).cpu().numpy()


def _wide_cases(rng, count):
    """Random and degenerate int64 point sets over the whole wide range."""
    for t in range(count):
        n = int(rng.integers(3, 700))
        kind = t % 8
        if kind == 0:    # uniform over the full box
            p = np.column_stack([rng.integers(-XY, XY, size=(n, 2), endpoint=True),
                                 rng.integers(-Z, Z, size=n, endpoint=True)])
        elif kind == 1:  # a small lattice blown up by powers of two: many ties
            q = rng.integers(0, 4, size=(n, 3))
            p = q * np.array([1 << 28, 1 << 28, 1 << 40])
        elif kind == 2:  # lifted points (Delaunay): all on the paraboloid
            xy = rng.integers(-(1 << 20), 1 << 20, size=(n, 2), endpoint=True)
            p = np.column_stack([xy, (xy * xy).sum(axis=1)])
        elif kind == 3:  # all x equal, at the bound
            p = np.column_stack([np.full(n, XY), rng.integers(-XY, XY, size=n, endpoint=True),
                                 rng.integers(-Z, Z, size=n, endpoint=True)])
        elif kind == 4:  # coplanar (z a linear function of x, y)
            xy = rng.integers(-(1 << 20), 1 << 20, size=(n, 2), endpoint=True)
            p = np.column_stack([xy, 3 * xy[:, 0] - 5 * xy[:, 1]])
        elif kind == 5:  # duplicates of a few extreme corners
            c = np.array([[sx * XY, sy * XY, sz * Z] for sx in (-1, 1) for sy in (-1, 1)
                          for sz in (-1, 1)])
            p = c[rng.integers(0, 8, size=n)]
        elif kind == 6:  # near-sphere with large radius in z
            g = rng.normal(size=(n, 3))
            g /= np.linalg.norm(g, axis=1, keepdims=True)
            p = np.rint(g * np.array([XY - 1, XY - 1, Z - 1])).astype(np.int64)
        else:            # narrow coordinates (the standard range) through the wide path
            p = rng.integers(-(1 << 20), 1 << 20, size=(n, 3), endpoint=True)
        yield t, np.ascontiguousarray(p.astype(np.int64))


def test_wide_parity(H, ws, strategy):
    rng = np.random.default_rng(30)
    for t, p in _wide_cases(rng, 64):
        say("wide case", strategy, t, "n", len(p))
        assert same(wide_faces(H, ws, p), oracle.hull_wide(p)), t
        if t % 4 == 0:
            assert same(wide_faces(H, ws, p, lower_only=True),
                        oracle.hull_wide(p, lower_only=True)), t


@pytest.mark.parametrize("n", [3, 4, 33, 1025, 4097, 20000])
def test_wide_ragged_sizes(H, ws, n):
    rng = np.random.default_rng(n + 1)
    p = np.column_stack([rng.integers(-XY, XY, size=(n, 2), endpoint=True),
                         rng.integers(-Z, Z, size=n, endpoint=True)]).astype(np.int64)
    say("wide ragged n", n)
    assert same(wide_faces(H, ws, p), oracle.hull_wide(p))


def test_wide_agrees_with_standard(H, ws):
    """On standard-range input both entry points give the oracle's faces."""
    import torch
    rng = np.random.default_rng(31)
    p = workloads.cube(rng, 5000, 1 << 29)
    say("wide vs standard", len(p))
    g = H.hull_sync(torch.from_numpy(p).cuda(), ws=ws).cpu().numpy()
    w = wide_faces(H, ws, p)
    assert same(g, w) and same(w, oracle.hull(p))


def test_wide_range_error(H, ws):
    import torch
    rng = np.random.default_rng(32)
    base = np.column_stack([rng.integers(-XY, XY, size=(500, 2), endpoint=True),
                            rng.integers(-Z, Z, size=500, endpoint=True)]).astype(np.int64)
    for col, bad in ((0, XY + 1), (1, -XY - 1), (2, Z + 1), (2, -Z - 1)):
        p = base.copy()
        p[211, col] = bad
        say("wide range error", col, bad)
        with pytest.raises(H.HullError) as e:
            H.hull_wide(torch.from_numpy(p).cuda(), ws=ws)
        assert e.value.code == H.HULL_ERANGE
    p = base.copy()
    p[7] = [XY, -XY, -Z]
    p[8] = [-XY, XY, Z]
    say("wide range edge")
    assert same(wide_faces(H, ws, p), oracle.hull_wide(p))


def _float_cases(rng):
    n = 900
    yield "unit cube", rng.uniform(-1, 1, size=(n, 3))
    yield "mixed magnitudes", rng.normal(size=(n, 3)) * np.exp2(rng.integers(-30, 30, size=(n, 1)))
    yield "half-integer ties", (rng.integers(-64, 64, size=(n, 3)) + 0.5) * 2.0 ** -10
    yield "tiny and subnormal", rng.normal(size=(n, 3)) * 2.0 ** -140
    yield "zeros and signed zeros", np.concatenate(
        [rng.uniform(-3, 3, size=(n - 20, 3)), np.zeros((10, 3)), -np.zeros((10, 3))])
    yield "huge", rng.normal(size=(n, 3)) * 2.0 ** 120
    yield "few distinct", rng.integers(-2, 3, size=(n, 3)).astype(np.float64) * 1.5


@pytest.mark.parametrize("bits", [1, 8, 20, 29, 30])
def test_f32_parity(H, ws, bits):
    rng = np.random.default_rng(40 + bits)
    for name, p in _float_cases(rng):
        p = p.astype(np.float32)
        say("f32", bits, name)
        assert same(f32_faces(H, ws, p, bits), floatin.hull_f32(p, bits)), name
        assert same(f32_faces(H, ws, p, bits, lower_only=True),
                    floatin.hull_f32(p, bits, lower_only=True)), name


def test_f32_strategies(H, ws, strategy):
    rng = np.random.default_rng(50)
    p = (rng.normal(size=(6000, 3)) * 3.0).astype(np.float32)
    say("f32 strategy", strategy)
    assert same(f32_faces(H, ws, p, 30), floatin.hull_f32(p, 30))


def test_f32_errors(H, ws):
    import torch
    p = np.random.default_rng(51).normal(size=(100, 3)).astype(np.float32)
    for bad in (np.nan, np.inf, -np.inf):
        q = p.copy()
        q[37, 1] = bad
        say("f32 non-finite", bad)
        with pytest.raises(H.HullError) as e:
            H.hull_f32(torch.from_numpy(q).cuda(), 30, ws=ws)
        assert e.value.code == H.HULL_ERANGE
    for bits in (0, 31):
        with pytest.raises(H.HullError) as e:
            H.hull_f32(torch.from_numpy(p).cuda(), bits, ws=ws)
        assert e.value.code == H.HULL_EINVAL
    say("f32 small n")
    for n in (0, 1, 2):
        assert f32_faces(H, ws, p[:n], 30).shape == (0, 3)
    assert same(f32_faces(H, ws, p[:3], 30), floatin.hull_f32(p[:3], 30))


def test_f32_full_size_digest(H, ws):
    path = os.path.join(GOLDEN, "float_ball.json")
    rec = json.load(open(path))
    p = workloads.float_ball()
    assert hashlib.sha256(np.ascontiguousarray(p, dtype="<f4").tobytes()).hexdigest() == \
        rec["input_sha256"]
    say("float_ball lower", len(p))
    gl = f32_faces(H, ws, p, rec["bits"], lower_only=True)
    assert len(gl) == rec["F_lower"]
    assert hashlib.sha256(validate.canonical(gl).astype("<i4").tobytes()).hexdigest() == \
        rec["sha256_lower"]
    say("float_ball full", len(p))
    g = f32_faces(H, ws, p, rec["bits"])
    assert len(g) == rec["F"]
    assert hashlib.sha256(validate.canonical(g).astype("<i4").tobytes()).hexdigest() == \
        rec["sha256_full"]
    assert validate.euler_ok(g) and validate.manifold_ok(g)

"""The C ABI on the host: every function declared in include/hull3d.h is
exported by the built library, and argument errors are reported
synchronously without touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1205_1171_amd import hull

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(hull.SO):
        from paper_1205_1171_amd import build
        build.build()
    return hull.lib()


def declared_functions():
    names = []
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(hull_[A-Za-z0-9_]+)\s*\(",
                                src, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert "hull_full" in names and "hull_lower" in names
    for n in names:
        assert hasattr(L, n), n


def test_strerror(L):
    for code in (0, -1, -2, -3, -4, -5):
        assert L.hull_strerror(code)
    assert b"unknown" in L.hull_strerror(77)


def test_workspace_bytes(L):
    assert hull.workspace_bytes(0) > 0
    a, b = hull.workspace_bytes(1000), hull.workspace_bytes(100000)
    assert b > a
    out = ctypes.c_size_t(0)
    assert L.hull_workspace_bytes(-1, 0, ctypes.byref(out)) == hull.HULL_EINVAL
    assert L.hull_workspace_bytes((1 << 26) + 1, 0, ctypes.byref(out)) == hull.HULL_EINVAL
    assert L.hull_workspace_bytes(10, 0, None) == hull.HULL_EINVAL


def test_argument_errors_are_synchronous(L):
    P = ctypes.c_void_p
    fake = P(0x1000)  # never dereferenced: every call below fails its checks first
    info = P(0x2000)
    ws = hull.workspace_bytes(100)
    for fn in (L.hull_lower, L.hull_full):
        assert fn(None, 100, fake, 200, info, fake, ws, None) == hull.HULL_EINVAL
        assert fn(fake, -1, fake, 200, info, fake, ws, None) == hull.HULL_EINVAL
        assert fn(fake, 100, fake, 199, info, fake, ws, None) == hull.HULL_EINVAL
        assert fn(fake, 100, None, 200, info, fake, ws, None) == hull.HULL_EINVAL
        assert fn(fake, 100, fake, 200, None, fake, ws, None) == hull.HULL_EINVAL
        assert fn(fake, 100, fake, 200, info, None, ws, None) == hull.HULL_EINVAL
        assert fn(fake, 100, fake, 200, info, fake, ws - 1, None) == hull.HULL_EWORKSPACE
        assert fn(fake, (1 << 26) + 1, fake, 1 << 28, info, fake, 1 << 40, None) == hull.HULL_EINVAL
    assert L.hull_movies(fake, 100, 2, 1, fake, fake, fake, info, fake, ws, None) == hull.HULL_EINVAL
    assert L.hull_movies(fake, 0, 0, 1, fake, fake, fake, info, fake, ws, None) == hull.HULL_EINVAL


def test_volume_area_argument_errors(L):
    P = ctypes.c_void_p
    fake = P(0x1000)
    assert L.hull_volume_area_fwd(fake, fake, fake, fake, -1, fake, fake, None) == hull.HULL_EINVAL
    assert L.hull_volume_area_fwd(None, fake, fake, fake, 2, fake, fake, None) == hull.HULL_EINVAL
    assert L.hull_volume_area_fwd(fake, fake, fake, fake, 2, None, fake, None) == hull.HULL_EINVAL
    assert L.hull_volume_area_fwd(None, None, None, None, 0, None, None, None) == hull.HULL_OK
    assert L.hull_volume_area_bwd(fake, fake, fake, fake, -3, fake, fake, fake, None) == hull.HULL_EINVAL
    assert L.hull_volume_area_bwd(fake, fake, None, fake, 2, fake, fake, fake, None) == hull.HULL_EINVAL
    assert L.hull_volume_area_bwd(fake, fake, fake, fake, 2, fake, fake, None, None) == hull.HULL_EINVAL


def test_batched_argument_errors(L):
    import numpy as np
    P = ctypes.c_void_p
    fake = P(0x1000)
    info = P(0x2000)

    def call(h_off, H=None, cap=None, ws=None, d_off=fake, faces=fake, face_off=fake):
        h_off = np.asarray(h_off, dtype=np.int64)
        H = len(h_off) - 1 if H is None else H
        N = int(h_off[-1]) if len(h_off) else 0
        cap = 2 * N if cap is None else cap
        if ws is None:
            ws = hull.workspace_bytes_batched(max(N, 0), max(H, 1))
        return L.hull_full_batched(fake, d_off, P(h_off.ctypes.data), H, faces, cap, face_off, info,
                                   fake, ws, None, None)

    assert call([0, 10, 30], H=0) == hull.HULL_EINVAL
    assert call([1, 10, 30]) == hull.HULL_EINVAL  # offsets[0] != 0
    assert call([0, 20, 10]) == hull.HULL_EINVAL  # decreasing
    assert call([0, 10, 30], cap=59) == hull.HULL_EINVAL
    assert call([0, 10, 30], d_off=None) == hull.HULL_EINVAL
    assert call([0, 10, 30], faces=None) == hull.HULL_EINVAL
    assert call([0, 10, 30], face_off=None) == hull.HULL_EINVAL
    assert call([0, (1 << 26) + 1], ws=1 << 40) == hull.HULL_EINVAL  # one cloud too large
    ws = hull.workspace_bytes_batched(30, 2)
    assert call([0, 10, 30], ws=ws - 1) == hull.HULL_EWORKSPACE
    out = ctypes.c_size_t(0)
    assert L.hull_workspace_bytes_batched(10, 0, ctypes.byref(out)) == hull.HULL_EINVAL
    assert L.hull_workspace_bytes_batched(-1, 1, ctypes.byref(out)) == hull.HULL_EINVAL
    # more hulls need more schedule space
    assert hull.workspace_bytes_batched(1000, 100) > hull.workspace_bytes_batched(1000, 1)


def test_adjacency_argument_errors(L):
    P = ctypes.c_void_p
    fake = P(0x1000)
    out = ctypes.c_size_t(0)
    assert L.hull_adjacency_workspace_bytes(-1, ctypes.byref(out)) == hull.HULL_EINVAL
    assert L.hull_adjacency_workspace_bytes(100, ctypes.byref(out)) == hull.HULL_OK
    ws = out.value
    assert ws >= 16 * 600
    f = L.hull_face_adjacency
    assert f(None, 100, None, None, 1, fake, fake, fake, ws, None) == hull.HULL_EINVAL
    assert f(fake, 100, None, None, 1, None, fake, fake, ws, None) == hull.HULL_EINVAL
    assert f(fake, 100, None, None, 1, fake, None, fake, ws, None) == hull.HULL_EINVAL
    assert f(fake, 100, fake, None, 1, fake, fake, fake, ws, None) == hull.HULL_EINVAL
    assert f(fake, 100, fake, fake, 0, fake, fake, fake, ws, None) == hull.HULL_EINVAL
    assert f(fake, 100, None, None, 1, fake, fake, fake, ws - 1, None) == hull.HULL_EWORKSPACE


def test_delaunay_argument_errors(L):
    P = ctypes.c_void_p
    fake = P(0x1000)
    out = ctypes.c_size_t(0)
    assert L.hull_delaunay_workspace_bytes(100, ctypes.byref(out)) == hull.HULL_OK
    assert out.value > hull.workspace_bytes(100)
    ws = out.value
    f = L.hull_delaunay
    assert f(None, 100, fake, 200, fake, fake, ws, None) == hull.HULL_EINVAL
    assert f(fake, 100, fake, 199, fake, fake, ws, None) == hull.HULL_EINVAL
    assert f(fake, -1, fake, 200, fake, fake, ws, None) == hull.HULL_EINVAL
    assert f(fake, 100, fake, 200, None, fake, ws, None) == hull.HULL_EINVAL
    assert f(fake, 100, fake, 200, fake, fake, ws - 1, None) == hull.HULL_EWORKSPACE


def test_schedule_defaults(L, monkeypatch):
    """Built-in defaults, the environment overrides, and the number of
    LDS-staged levels reported in fused_levels."""
    for k in ("HULL_SERIAL_LEVELS", "HULL_WALK_SEGMENT", "HULL_WAVE_LEVEL", "HULL_WAVE_LANES",
              "HULL_LDS_LEVELS", "HULL_WAVE_LANES_MAX"):
        monkeypatch.delenv(k, raising=False)
    s = hull.schedule_defaults()
    assert (s.serial_levels, s.walk_segment, s.wave_from, s.wave_lanes) == (10, 4, 8, 8)
    assert s.wave_lanes_max == 64
    assert 0 <= s.fused_levels <= s.serial_levels
    assert s.fused_levels == 3
    monkeypatch.setenv("HULL_LDS_LEVELS", "9")  # at most 4 levels stage points in LDS
    assert hull.schedule_defaults().fused_levels == 4
    monkeypatch.setenv("HULL_LDS_LEVELS", "0")
    assert hull.schedule_defaults().fused_levels == 0
    monkeypatch.delenv("HULL_LDS_LEVELS")
    monkeypatch.setenv("HULL_WAVE_LEVEL", "2")  # raised above the LDS-staged levels (3), to 4
    assert hull.schedule_defaults().wave_from == 4
    monkeypatch.setenv("HULL_LDS_LEVELS", "4")
    assert hull.schedule_defaults().wave_from == 5
    monkeypatch.delenv("HULL_LDS_LEVELS")
    monkeypatch.setenv("HULL_WAVE_LEVEL", "-1")
    assert hull.schedule_defaults().wave_from == 0
    monkeypatch.delenv("HULL_WAVE_LEVEL")
    monkeypatch.setenv("HULL_WAVE_LANES", "64")
    assert hull.schedule_defaults().wave_lanes == 64
    monkeypatch.setenv("HULL_WAVE_LANES_MAX", "8")  # never below the first level's lanes
    assert hull.schedule_defaults().wave_lanes_max == 64
    monkeypatch.setenv("HULL_WAVE_LANES", "16")
    monkeypatch.setenv("HULL_WAVE_LANES_MAX", "20")  # rounded down to a lane count
    assert hull.schedule_defaults().wave_lanes_max == 16
    monkeypatch.delenv("HULL_WAVE_LANES_MAX")
    monkeypatch.delenv("HULL_WAVE_LANES")
    monkeypatch.setenv("HULL_SERIAL_LEVELS", "12")
    monkeypatch.setenv("HULL_WALK_SEGMENT", "32")
    s = hull.schedule_defaults()
    assert (s.serial_levels, s.walk_segment) == (12, 32)
    monkeypatch.setenv("HULL_WALK_SEGMENT", "2")  # below the minimum of 4
    assert hull.schedule_defaults().walk_segment == 4
    assert L.hull_schedule_defaults(None) == hull.HULL_EINVAL


def test_adjacency_face_limit(L):
    """Half-edge ids are int32: F above (2^31 - 3) / 3 is refused."""
    out = ctypes.c_size_t(0)
    fmax = ((1 << 31) - 3) // 3
    assert L.hull_adjacency_workspace_bytes(fmax, ctypes.byref(out)) == hull.HULL_OK
    assert L.hull_adjacency_workspace_bytes(fmax + 1, ctypes.byref(out)) == hull.HULL_EINVAL
    P = ctypes.c_void_p
    fake = P(0x1000)
    assert L.hull_face_adjacency(fake, fmax + 1, None, None, 1, fake, fake, fake, 1 << 40,
                                 None) == hull.HULL_EINVAL


def test_workspace_kinds(L):
    out = ctypes.c_size_t(0)
    n = 100000
    sizes = []
    for flags in (hull.WS_STANDARD, hull.WS_WIDE, hull.WS_F32):
        assert L.hull_workspace_bytes(n, flags, ctypes.byref(out)) == hull.HULL_OK
        sizes.append(out.value)
    # the wide points take 32 bytes instead of 16; the float entry adds its rows
    assert sizes[1] >= sizes[0] + 16 * n and sizes[2] >= sizes[1] + 24 * n
    for flags in (-1, 3, 77):
        assert L.hull_workspace_bytes(n, flags, ctypes.byref(out)) == hull.HULL_EINVAL
    assert L.hull_delaunay_workspace_bytes(n, ctypes.byref(out)) == hull.HULL_OK
    assert out.value >= sizes[1] + 24 * n


def test_wide_and_f32_argument_errors(L):
    P = ctypes.c_void_p
    fake = P(0x1000)
    info = P(0x2000)
    out = ctypes.c_size_t(0)
    L.hull_workspace_bytes(100, hull.WS_WIDE, ctypes.byref(out))
    wsw = out.value
    L.hull_workspace_bytes(100, hull.WS_F32, ctypes.byref(out))
    wsf = out.value
    for fn in (L.hull_lower_wide, L.hull_full_wide):
        assert fn(None, 100, fake, 200, info, fake, wsw, None) == hull.HULL_EINVAL
        assert fn(fake, 100, fake, 199, info, fake, wsw, None) == hull.HULL_EINVAL
        assert fn(fake, 100, fake, 200, None, fake, wsw, None) == hull.HULL_EINVAL
        assert fn(fake, 100, fake, 200, info, fake, wsw - 1, None) == hull.HULL_EWORKSPACE
        assert fn(fake, (1 << 26) + 1, fake, 1 << 28, info, fake, 1 << 40, None) == hull.HULL_EINVAL
    for fn in (L.hull_lower_f32, L.hull_full_f32):
        assert fn(fake, 100, 0, fake, 200, info, fake, wsf, None) == hull.HULL_EINVAL
        assert fn(fake, 100, 31, fake, 200, info, fake, wsf, None) == hull.HULL_EINVAL
        assert fn(None, 100, 30, fake, 200, info, fake, wsf, None) == hull.HULL_EINVAL
        assert fn(fake, 100, 30, fake, 199, info, fake, wsf, None) == hull.HULL_EINVAL
        assert fn(fake, 100, 30, fake, 200, info, fake, wsf - 1, None) == hull.HULL_EWORKSPACE


def test_workspace_limits(L):
    """Workspace per point stays below 1 KiB (n = 2^24 under 16 GiB); the
    batch limit is 2^28 points, whose workspace fits 288 GB."""
    out = ctypes.c_size_t(0)
    n = 1 << 24
    assert L.hull_workspace_bytes(n, 0, ctypes.byref(out)) == hull.HULL_OK
    assert out.value < 1024 * n
    assert L.hull_workspace_bytes_batched(1 << 28, 10000, ctypes.byref(out)) == hull.HULL_OK
    assert out.value < 288e9
    assert L.hull_workspace_bytes_batched((1 << 28) + 1, 10000, ctypes.byref(out)) == hull.HULL_EINVAL
    assert L.hull_workspace_bytes((1 << 26), 0, ctypes.byref(out)) == hull.HULL_OK
    assert out.value < 288e9


def test_schedule_struct_matches_header():
    """The binding's hull_schedule_t has the header's fields, in its order,
    all int32 (the library reads them by offset)."""
    src = open(os.path.join(ROOT, "include", "hull3d.h")).read()
    body = re.search(r"typedef struct hull_schedule_t \{(.*?)\} hull_schedule_t;", src, flags=re.S)
    assert body
    fields = re.findall(r"int32_t\s+([a-z_]+);", body.group(1))
    assert [f for f, _ in hull.Schedule._fields_] == fields
    assert all(t is ctypes.c_int32 for _, t in hull.Schedule._fields_)
    assert ctypes.sizeof(hull.Schedule) == 4 * len(fields)

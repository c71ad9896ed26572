"""Python binding of the C ABI in ``include/hull3d.h`` (ctypes).

Argument marshalling only: every step of the hull runs in the HIP library.
PyTorch supplies device memory and the current stream.  If the library has
not been built, every call raises: there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libhull3d.so")

HULL_OK = 0
HULL_EINVAL = -1
HULL_EWORKSPACE = -2
HULL_ERANGE = -3
HULL_EHIP = -4
HULL_EINTERNAL = -5

_lib = None


class Schedule(ctypes.Structure):
    """hull_schedule_t: merge schedule of a batched call (-1 / 0 = default)."""
    _fields_ = [("serial_levels", ctypes.c_int32), ("walk_segment", ctypes.c_int32),
                ("fused_levels", ctypes.c_int32), ("wave_from", ctypes.c_int32),
                ("wave_lanes", ctypes.c_int32), ("wave_lanes_max", ctypes.c_int32)]

    def __init__(self, serial_levels=-1, walk_segment=0, fused_levels=-1, wave_from=0,
                 wave_lanes=0, wave_lanes_max=0):
        super().__init__(int(serial_levels), int(walk_segment), int(fused_levels), int(wave_from),
                         int(wave_lanes), int(wave_lanes_max))


class HullError(RuntimeError):
    def __init__(self, code, where=""):
        msg = _strerror(code) if _lib is not None else str(code)
        if code == HULL_EHIP and _lib is not None:
            msg += f", hipError_t {_lib.hull_last_hip_error()}"
        super().__init__(f"{where}: {msg} ({code})")
        self.code = code


def _strerror(code):
    return _lib.hull_strerror(code).decode()


def lib():
    """The loaded HIP library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(SO):
        raise RuntimeError(f"HIP library not built: {SO} (run __graft_entry__.build())")
    # torch first: its HIP runtime (libamdhip64.so.7) is then the one the
    # library binds to.  Loaded the other way round, the process would hold
    # two HIP runtimes and the library's would find no device.
    import torch  # noqa: F401
    L = ctypes.CDLL(SO)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    sz = ctypes.c_size_t
    L.hull_strerror.argtypes = [i32]
    L.hull_strerror.restype = ctypes.c_char_p
    L.hull_last_hip_error.argtypes = []
    L.hull_last_hip_error.restype = i32
    L.hull_workspace_bytes.argtypes = [i64, i32, ctypes.POINTER(sz)]
    L.hull_workspace_bytes.restype = i32
    for f in (L.hull_lower, L.hull_full):
        f.argtypes = [P, i64, P, i64, P, P, sz, P]
        f.restype = i32
    for f in (L.hull_lower_wide, L.hull_full_wide):
        f.argtypes = [P, i64, P, i64, P, P, sz, P]
        f.restype = i32
    for f in (L.hull_lower_f32, L.hull_full_f32):
        f.argtypes = [P, i64, i32, P, i64, P, P, sz, P]
        f.restype = i32
    L.hull_full_timed.argtypes = [P, i64, P, i64, P, P, sz, P, P, i32]
    L.hull_full_timed.restype = i32
    L.hull_workspace_bytes_batched.argtypes = [i64, i64, ctypes.POINTER(sz)]
    L.hull_workspace_bytes_batched.restype = i32
    L.hull_full_batched.argtypes = [P, P, P, i64, P, i64, P, P, P, sz, ctypes.POINTER(Schedule), P]
    L.hull_full_batched.restype = i32
    L.hull_schedule_defaults.argtypes = [ctypes.POINTER(Schedule)]
    L.hull_schedule_defaults.restype = i32
    L.hull_adjacency_workspace_bytes.argtypes = [i64, ctypes.POINTER(sz)]
    L.hull_adjacency_workspace_bytes.restype = i32
    L.hull_face_adjacency.argtypes = [P, i64, P, P, i64, P, P, P, sz, P]
    L.hull_face_adjacency.restype = i32
    L.hull_delaunay_workspace_bytes.argtypes = [i64, ctypes.POINTER(sz)]
    L.hull_delaunay_workspace_bytes.restype = i32
    L.hull_delaunay.argtypes = [P, i64, P, i64, P, P, sz, P]
    L.hull_delaunay.restype = i32
    L.hull_movies.argtypes = [P, i64, i32, i32, P, P, P, P, P, sz, P]
    L.hull_movies.restype = i32
    L.hull_volume_area_fwd.argtypes = [P, P, P, P, i32, P, P, P]
    L.hull_volume_area_fwd.restype = i32
    L.hull_volume_area_bwd.argtypes = [P, P, P, P, i32, P, P, P, P]
    L.hull_volume_area_bwd.restype = i32
    _lib = L
    return L


def exported_symbols():
    """Names declared in include/hull3d.h that the library exports."""
    L = lib()
    names = ["hull_strerror", "hull_last_hip_error", "hull_workspace_bytes", "hull_lower", "hull_full", "hull_full_timed",
             "hull_lower_wide", "hull_full_wide", "hull_lower_f32", "hull_full_f32",
             "hull_workspace_bytes_batched", "hull_full_batched", "hull_schedule_defaults",
             "hull_movies", "hull_adjacency_workspace_bytes", "hull_face_adjacency",
             "hull_delaunay_workspace_bytes", "hull_delaunay",
             "hull_volume_area_fwd", "hull_volume_area_bwd"]
    return [n for n in names if hasattr(L, n)]


WS_STANDARD, WS_WIDE, WS_F32 = 0, 1, 2


def workspace_bytes(n, flags=WS_STANDARD):
    out = ctypes.c_size_t(0)
    rc = lib().hull_workspace_bytes(int(n), int(flags), ctypes.byref(out))
    if rc:
        raise HullError(rc, "hull_workspace_bytes")
    return out.value


def schedule_defaults():
    """The schedule the library uses for calls that pass none."""
    out = Schedule()
    rc = lib().hull_schedule_defaults(ctypes.byref(out))
    if rc:
        raise HullError(rc, "hull_schedule_defaults")
    return out


def workspace_bytes_batched(total_points, H):
    out = ctypes.c_size_t(0)
    rc = lib().hull_workspace_bytes_batched(int(total_points), int(H), ctypes.byref(out))
    if rc:
        raise HullError(rc, "hull_workspace_bytes_batched")
    return out.value


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _on(stream):
    """Context that makes ``stream`` current (no-op for None), so that the
    temporaries a wrapper allocates and the copies it makes are ordered on
    the stream its kernels run on (the caching allocator then also keeps
    them until that stream is done with them)."""
    import contextlib
    import torch
    return contextlib.nullcontext() if stream is None else torch.cuda.stream(stream)


def _check_points(xyz):
    import torch
    if not (isinstance(xyz, torch.Tensor) and xyz.is_cuda and xyz.dtype == torch.int32):
        raise TypeError("points must be a CUDA int32 tensor")
    if xyz.dim() != 2 or xyz.shape[1] != 3 or not xyz.is_contiguous():
        raise ValueError("points must be a contiguous [n, 3] tensor")


class Workspace:
    """Reusable device workspace (grows on demand)."""

    def __init__(self, device=None):
        self.buf = None
        self.device = device

    def get(self, nbytes, device):
        import torch
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


def hull(xyz, lower_only=False, ws=None, faces=None, info=None, stream=None):
    """Faces (device int32 [cap, 3]) and info (device int64 [2]: status, F).

    Asynchronous: the first info[1] rows of ``faces`` are valid once the
    stream reaches this point.  Use :func:`hull_sync` for a checked result."""
    _check_points(xyz)
    with _on(stream):
        return _hull(xyz, lower_only, ws, faces, info)


def _hull(xyz, lower_only, ws, faces, info):
    import torch
    n = xyz.shape[0]
    dev = xyz.device
    cap = max(2 * n, 1)
    if faces is None:
        faces = torch.empty((cap, 3), dtype=torch.int32, device=dev)
    if info is None:
        info = torch.empty(2, dtype=torch.int64, device=dev)
    nb = workspace_bytes(n)
    wbuf = (ws or Workspace()).get(nb, dev)
    fn = lib().hull_lower if lower_only else lib().hull_full
    rc = fn(ctypes.c_void_p(xyz.data_ptr()), n, ctypes.c_void_p(faces.data_ptr()), faces.shape[0],
            ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(wbuf.data_ptr()), wbuf.numel(),
            _stream(None))
    if rc:
        raise HullError(rc, "hull_lower" if lower_only else "hull_full")
    return faces, info


def hull_sync(xyz, lower_only=False, ws=None):
    """Blocking call: the face tensor [F, 3] on the device (checked status)."""
    faces, info = hull(xyz, lower_only=lower_only, ws=ws)
    st, F = (int(v) for v in info.cpu())
    if st:
        raise HullError(st, "device")
    return faces[:F]


def hull_wide(xyz, lower_only=False, ws=None, stream=None):
    """Blocking hull of int64 points [n, 3] on the wide range (|x|, |y| <=
    2^30, |z| <= 2^42): the face tensor [F, 3] on the device."""
    import torch
    if not (isinstance(xyz, torch.Tensor) and xyz.is_cuda and xyz.dtype == torch.int64):
        raise TypeError("points must be a CUDA int64 tensor")
    if xyz.dim() != 2 or xyz.shape[1] != 3 or not xyz.is_contiguous():
        raise ValueError("points must be a contiguous [n, 3] tensor")
    with _on(stream):
        n = xyz.shape[0]
        dev = xyz.device
        cap = max(2 * n, 1)
        faces = torch.empty((cap, 3), dtype=torch.int32, device=dev)
        info = torch.empty(2, dtype=torch.int64, device=dev)
        wbuf = (ws or Workspace()).get(workspace_bytes(n, WS_WIDE), dev)
        fn = lib().hull_lower_wide if lower_only else lib().hull_full_wide
        rc = fn(ctypes.c_void_p(xyz.data_ptr()), n, ctypes.c_void_p(faces.data_ptr()), cap,
                ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(wbuf.data_ptr()), wbuf.numel(),
                _stream(None))
        if rc:
            raise HullError(rc, "hull_lower_wide" if lower_only else "hull_full_wide")
        st, F = (int(v) for v in info.cpu())
    if st:
        raise HullError(st, "device")
    return faces[:F]


def hull_f32(p, bits=30, lower_only=False, ws=None, stream=None):
    """Blocking hull of float32 points [n, 3] snapped to the lattice of
    ``bits`` bits (scale 2^(bits - E), E the least integer with max |c| <=
    2^E; round to nearest, ties to even): the face tensor [F, 3]."""
    import torch
    if not (isinstance(p, torch.Tensor) and p.is_cuda and p.dtype == torch.float32):
        raise TypeError("points must be a CUDA float32 tensor")
    if p.dim() != 2 or p.shape[1] != 3 or not p.is_contiguous():
        raise ValueError("points must be a contiguous [n, 3] tensor")
    with _on(stream):
        n = p.shape[0]
        dev = p.device
        cap = max(2 * n, 1)
        faces = torch.empty((cap, 3), dtype=torch.int32, device=dev)
        info = torch.empty(2, dtype=torch.int64, device=dev)
        wbuf = (ws or Workspace()).get(workspace_bytes(n, WS_F32), dev)
        fn = lib().hull_lower_f32 if lower_only else lib().hull_full_f32
        rc = fn(ctypes.c_void_p(p.data_ptr()), n, int(bits), ctypes.c_void_p(faces.data_ptr()),
                cap, ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(wbuf.data_ptr()),
                wbuf.numel(), _stream(None))
        if rc:
            raise HullError(rc, "hull_lower_f32" if lower_only else "hull_full_f32")
        st, F = (int(v) for v in info.cpu())
    if st:
        raise HullError(st, "device")
    return faces[:F]


def hull_batched(xyz, offsets, schedule=None, ws=None, faces=None, stream=None):
    """Full hulls of H clouds in one call: cloud h is rows [offsets[h],
    offsets[h+1]) of ``xyz``.  Returns (faces [cap, 3], face_offsets [H + 1],
    info [2]) on the device; the faces of cloud h are rows
    [face_offsets[h], face_offsets[h+1]), indices local to the cloud.
    Asynchronous, like :func:`hull`."""
    _check_points(xyz)
    with _on(stream):
        return _hull_batched(xyz, offsets, schedule, ws, faces)


def _hull_batched(xyz, offsets, schedule, ws, faces):
    import torch
    h_off = torch.as_tensor(offsets, dtype=torch.int64).cpu().contiguous()
    H = h_off.numel() - 1
    if H < 1 or int(h_off[-1]) != xyz.shape[0]:
        raise ValueError("offsets must have H + 1 >= 2 entries ending at the point count")
    dev = xyz.device
    d_off = h_off.to(dev)
    n = xyz.shape[0]
    cap = max(2 * n, 1)
    if faces is None:
        faces = torch.empty((cap, 3), dtype=torch.int32, device=dev)
    face_off = torch.empty(H + 1, dtype=torch.int64, device=dev)
    info = torch.empty(2, dtype=torch.int64, device=dev)
    wbuf = (ws or Workspace()).get(workspace_bytes_batched(n, H), dev)
    sc = ctypes.byref(schedule) if schedule is not None else None
    rc = lib().hull_full_batched(ctypes.c_void_p(xyz.data_ptr()), ctypes.c_void_p(d_off.data_ptr()),
                                 ctypes.c_void_p(h_off.data_ptr()), H,
                                 ctypes.c_void_p(faces.data_ptr()), faces.shape[0],
                                 ctypes.c_void_p(face_off.data_ptr()),
                                 ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(wbuf.data_ptr()),
                                 wbuf.numel(), sc, _stream(None))
    if rc:
        raise HullError(rc, "hull_full_batched")
    return faces, face_off, info


def hull_batched_sync(xyz, offsets, schedule=None, ws=None):
    """Blocking call: (faces [F, 3], face_offsets [H + 1]) on the device."""
    faces, face_off, info = hull_batched(xyz, offsets, schedule=schedule, ws=ws)
    st, F = (int(v) for v in info.cpu())
    if st:
        raise HullError(st, "device")
    return faces[:F], face_off


def face_adjacency(faces, face_off=None, pt_off=None, ws=None, stream=None):
    """Half-edge twins of face rows (device int32 [F, 3] -> device int32
    [F, 3]); face_off / pt_off: device int64 [H + 1] for a batch (vertex
    indices within each cloud).  Blocking: returns (adj, open_edges)."""
    with _on(stream):
        return _face_adjacency(faces, face_off, pt_off, ws)


def _face_adjacency(faces, face_off, pt_off, ws):
    import torch
    if not (isinstance(faces, torch.Tensor) and faces.is_cuda and faces.dtype == torch.int32):
        raise TypeError("faces must be a CUDA int32 tensor")
    faces = faces.contiguous()
    F = faces.shape[0]
    dev = faces.device
    adj = torch.empty((max(F, 1), 3), dtype=torch.int32, device=dev)
    info = torch.empty(2, dtype=torch.int64, device=dev)
    nb = ctypes.c_size_t(0)
    rc = lib().hull_adjacency_workspace_bytes(F, ctypes.byref(nb))
    if rc:
        raise HullError(rc, "hull_adjacency_workspace_bytes")
    wbuf = (ws or Workspace()).get(nb.value, dev)
    H = 1 if face_off is None else face_off.numel() - 1
    rc = lib().hull_face_adjacency(ctypes.c_void_p(faces.data_ptr()), F, _ptr(face_off),
                                   _ptr(pt_off), H, ctypes.c_void_p(adj.data_ptr()),
                                   ctypes.c_void_p(info.data_ptr()),
                                   ctypes.c_void_p(wbuf.data_ptr()), wbuf.numel(), _stream(None))
    if rc:
        raise HullError(rc, "hull_face_adjacency")
    st, open_edges = (int(v) for v in info.cpu())
    if st:
        raise HullError(st, "device")
    return adj[:F], open_edges


def delaunay(xy, ws=None, stream=None):
    """Delaunay triangles (device int32 [T, 3], counter-clockwise) of the
    CUDA int32 points xy [n, 2], |x|, |y| <= 2^20.  Blocking (checked)."""
    with _on(stream):
        return _delaunay(xy, ws)


def _delaunay(xy, ws):
    import torch
    if not (isinstance(xy, torch.Tensor) and xy.is_cuda and xy.dtype == torch.int32):
        raise TypeError("points must be a CUDA int32 tensor")
    if xy.dim() != 2 or xy.shape[1] != 2 or not xy.is_contiguous():
        raise ValueError("points must be a contiguous [n, 2] tensor")
    n = xy.shape[0]
    dev = xy.device
    cap = max(2 * n, 1)
    tris = torch.empty((cap, 3), dtype=torch.int32, device=dev)
    info = torch.empty(2, dtype=torch.int64, device=dev)
    nb = ctypes.c_size_t(0)
    rc = lib().hull_delaunay_workspace_bytes(n, ctypes.byref(nb))
    if rc:
        raise HullError(rc, "hull_delaunay_workspace_bytes")
    wbuf = (ws or Workspace()).get(nb.value, dev)
    rc = lib().hull_delaunay(ctypes.c_void_p(xy.data_ptr()), n, ctypes.c_void_p(tris.data_ptr()), cap,
                             ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(wbuf.data_ptr()),
                             wbuf.numel(), _stream(None))
    if rc:
        raise HullError(rc, "hull_delaunay")
    st, T = (int(v) for v in info.cpu())
    if st:
        raise HullError(st, "device")
    return tris[:T]


def movies(xyz, run, level, ws=None):
    """Movies after ``level`` merge levels: (events [E, 4] in rank terms,
    per-block lengths, rank -> input index), all copied to the host."""
    import torch
    _check_points(xyz)
    n = xyz.shape[0]
    dev = xyz.device
    ev = torch.zeros((2 * n, 4), dtype=torch.int32, device=dev)
    bl = torch.zeros(n, dtype=torch.int32, device=dev)
    order = torch.empty(n, dtype=torch.int32, device=dev)
    info = torch.empty(2, dtype=torch.int64, device=dev)
    nb = workspace_bytes(n)
    wbuf = (ws or Workspace()).get(nb, dev)
    rc = lib().hull_movies(ctypes.c_void_p(xyz.data_ptr()), n, int(run), int(level),
                           ctypes.c_void_p(ev.data_ptr()), ctypes.c_void_p(bl.data_ptr()),
                           ctypes.c_void_p(order.data_ptr()), ctypes.c_void_p(info.data_ptr()),
                           ctypes.c_void_p(wbuf.data_ptr()), wbuf.numel(), _stream(None))
    if rc:
        raise HullError(rc, "hull_movies")
    st = int(info[0].item())
    if st:
        raise HullError(st, "device")
    return ev.cpu().numpy(), bl.cpu().numpy(), order.cpu().numpy()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_volume_args(p, pt_off, faces, face_off):
    import torch
    for name, t, dt in (("p", p, torch.float32), ("pt_off", pt_off, torch.int64),
                        ("faces", faces, torch.int32), ("face_off", face_off, torch.int64)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
            raise TypeError(f"{name} must be a contiguous CUDA {dt} tensor")
        if t.device != p.device:
            raise ValueError(f"{name} is on {t.device}, points on {p.device}")
    if p.dim() != 2 or p.shape[1] != 3 or faces.dim() != 2 or faces.shape[1] != 3:
        raise ValueError("p and faces must be [N, 3] and [F, 3]")
    if pt_off.dim() != 1 or face_off.shape != pt_off.shape or pt_off.numel() < 2:
        raise ValueError("pt_off and face_off must both be [H + 1], H >= 1")


def volume_area_fwd(p, pt_off, faces, face_off, stream=None):
    """(V, A) per cloud, float32 device tensors [H]."""
    import torch
    _check_volume_args(p, pt_off, faces, face_off)
    H = pt_off.numel() - 1
    with _on(stream):
        V = torch.empty(H, dtype=torch.float32, device=p.device)
        A = torch.empty(H, dtype=torch.float32, device=p.device)
        rc = lib().hull_volume_area_fwd(_ptr(p), _ptr(pt_off), _ptr(faces), _ptr(face_off), H,
                                        _ptr(V), _ptr(A), _stream(None))
    if rc:
        raise HullError(rc, "hull_volume_area_fwd")
    return V, A


def volume_area_bwd(p, pt_off, faces, face_off, gV, gA, stream=None):
    """Gradient [N, 3] of sum(gV * V + gA * A) with respect to p (gV or gA
    may be None)."""
    import torch
    _check_volume_args(p, pt_off, faces, face_off)
    H = pt_off.numel() - 1
    for name, t in (("gV", gV), ("gA", gA)):  # None: that term has no gradient
        if t is not None and not (isinstance(t, torch.Tensor) and t.is_cuda
                                  and t.dtype == torch.float32 and t.is_contiguous()
                                  and t.numel() == H and t.device == p.device):
            raise TypeError(f"{name} must be None or a contiguous CUDA float32 tensor of {H} "
                            "entries")
    with _on(stream):
        g = torch.empty_like(p)
        rc = lib().hull_volume_area_bwd(_ptr(p), _ptr(pt_off), _ptr(faces), _ptr(face_off), H,
                                        _ptr(gV), _ptr(gA), _ptr(g), _stream(None))
    if rc:
        raise HullError(rc, "hull_volume_area_bwd")
    return g


class BatchedHull:
    """A fixed batch layout with its device buffers, for repeated calls of
    hull_full_batched on inputs of that layout (same offsets, same input
    buffer).  ``run`` launches on the current stream; ``capture`` records one
    call into a HIP graph (the library makes no allocation, copy, memset or
    host synchronisation, so the whole call is capturable) and ``replay``
    launches it."""

    def __init__(self, xyz, offsets, schedule=None):
        import torch
        _check_points(xyz)
        self.xyz = xyz
        self.h_off = torch.as_tensor(offsets, dtype=torch.int64).cpu().contiguous()
        self.H = self.h_off.numel() - 1
        if self.H < 1 or int(self.h_off[-1]) != xyz.shape[0]:
            raise ValueError("offsets must have H + 1 >= 2 entries ending at the point count")
        dev = xyz.device
        n = xyz.shape[0]
        self.d_off = self.h_off.to(dev)
        self.cap = max(2 * n, 1)
        self.faces = torch.empty((self.cap, 3), dtype=torch.int32, device=dev)
        self.face_off = torch.zeros(self.H + 1, dtype=torch.int64, device=dev)
        self.info = torch.zeros(2, dtype=torch.int64, device=dev)
        self.ws = torch.empty(max(workspace_bytes_batched(n, self.H), 256), dtype=torch.uint8,
                              device=dev)
        self.schedule = schedule
        self.graph = None

    def run(self, stream=None):
        sc = ctypes.byref(self.schedule) if self.schedule is not None else None
        rc = lib().hull_full_batched(
            ctypes.c_void_p(self.xyz.data_ptr()), ctypes.c_void_p(self.d_off.data_ptr()),
            ctypes.c_void_p(self.h_off.data_ptr()), self.H, ctypes.c_void_p(self.faces.data_ptr()),
            self.cap, ctypes.c_void_p(self.face_off.data_ptr()), ctypes.c_void_p(self.info.data_ptr()),
            ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(), sc, _stream(stream))
        if rc:
            raise HullError(rc, "hull_full_batched")

    def capture(self):
        import torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()  # warm-up outside the graph
        torch.cuda.current_stream().wait_stream(s)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def result(self):
        """Checked (faces [F, 3], face_offsets [H + 1]) after a call (blocking)."""
        st, F = (int(v) for v in self.info.cpu())
        if st:
            raise HullError(st, "device")
        return self.faces[:F], self.face_off

"""hull_full_noalloc (the entry point that allocates nothing: its scratch is
a fixed device array of the library) against hull_full, through the C ABI:
the same faces on two calls in a row, the second on a smaller input, and a
clear error for an input whose scratch would not fit."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import validate
from paper_1205_1171_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def same(a, b):
    a, b = validate.canonical(a), validate.canonical(b)
    return a.shape == b.shape and bool((a == b).all())


def _noalloc(L, x, n, faces, info, sptr):
    return L.hull_full_noalloc(ctypes.c_void_p(x.data_ptr()), n, ctypes.c_void_p(faces.data_ptr()),
                               faces.shape[0], ctypes.c_void_p(info.data_ptr()), sptr)


def test_noalloc_matches_hull_full():
    import torch
    from paper_1205_1171_amd import hull
    L = hull.lib()
    L.hull_full_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    L.hull_full_noalloc.restype = ctypes.c_int32
    rng = np.random.default_rng(77)
    sptr = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # the largest n whose workspace fits the 64 MiB array
    nmax = 1
    while hull.workspace_bytes(2 * nmax) <= (64 << 20):
        nmax *= 2
    lo, hi = nmax, 2 * nmax
    while hi - lo > 1:
        mid = (lo + hi) // 2
        if hull.workspace_bytes(mid) <= (64 << 20):
            lo = mid
        else:
            hi = mid
    nmax = lo
    say("noalloc nmax", nmax)
    for t, n in enumerate((nmax, 3000, 1000, 3)):
        p = workloads.sphere(rng, n, 1 << 16) if t % 2 else workloads.cube(rng, n, 1 << 29)
        x = torch.from_numpy(p).cuda()
        faces = torch.full((2 * n, 3), -7, dtype=torch.int32, device="cuda")
        info = torch.full((2,), -9, dtype=torch.int64, device="cuda")
        say("noalloc call", t, "n", n)
        assert _noalloc(L, x, n, faces, info, sptr) == hull.HULL_OK
        st, F = (int(v) for v in info.cpu())
        assert st == 0
        got = faces[:F].cpu().numpy()
        want = hull.hull_sync(x).cpu().numpy()
        assert same(got, want), (t, n)
        if n <= 3000:
            assert same(got, oracle.hull(p)), (t, n)
    # too large for the array: a synchronous error, nothing launched
    n = nmax + 1
    x = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
    faces = torch.empty((2 * n, 3), dtype=torch.int32, device="cuda")
    info = torch.zeros(2, dtype=torch.int64, device="cuda")
    assert _noalloc(L, x, n, faces, info, sptr) == hull.HULL_EWORKSPACE

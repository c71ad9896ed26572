"""GPU parity of hull_face_adjacency against the oracle's adjacency of the
same face rows (oracle/adjacency.py), on single hulls, ragged batches and the
full-size workloads.  Bit-exact (integer work): every twin equal."""
import numpy as np
import pytest

import oracle
from oracle import adjacency as adjmod
from paper_1205_1171_amd import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def H():
    import torch
    from paper_1205_1171_amd import hull
    assert torch.cuda.is_available()
    hull.lib()
    return hull


def test_single_hulls(H):
    import torch
    rng = np.random.default_rng(31)
    ws = H.Workspace()
    for t in range(30):
        n = int(rng.integers(3, 3000))
        p = [workloads.lattice(rng, n, 3), workloads.cube(rng, n, 1 << 20),
             workloads.sphere(rng, n, 1 << 12)][t % 3]
        faces = H.hull_sync(torch.from_numpy(np.ascontiguousarray(p)).cuda(), ws=ws)
        say("adjacency single", t, n, faces.shape[0])
        adj, open_edges = H.face_adjacency(faces, ws=ws)
        assert open_edges == 0
        assert (adj.cpu().numpy() == adjmod.adjacency(faces.cpu().numpy())).all(), t


def test_open_surface_and_errors(H):
    import torch
    p = workloads.cube(np.random.default_rng(2), 500, 1 << 20)
    faces = torch.from_numpy(oracle.hull(p).astype(np.int32)).cuda()
    adj, open_edges = H.face_adjacency(faces[1:])
    assert open_edges == 3
    assert (adj.cpu().numpy() == adjmod.adjacency(faces[1:].cpu().numpy())).all()
    with pytest.raises(H.HullError):  # a directed edge used twice
        H.face_adjacency(torch.cat([faces, faces[:1]]))
    with pytest.raises(H.HullError):  # a vertex index outside its cloud
        H.face_adjacency(faces, torch.tensor([0, len(faces)], device="cuda"),
                         torch.tensor([0, 10], device="cuda"))


def test_ragged_batch(H):
    import torch
    pts, off, _ = workloads.cfg4(H=300, lo=2.0, hi=12.0)
    x = torch.from_numpy(pts).cuda()
    f, fo = H.hull_batched_sync(x, off)
    say("adjacency batch", len(off) - 1, f.shape[0])
    adj, open_edges = H.face_adjacency(f, fo, torch.from_numpy(off).cuda())
    assert open_edges == 0
    assert (adj.cpu().numpy() == adjmod.adjacency(f.cpu().numpy(), fo.cpu().numpy())).all()


@pytest.mark.parametrize("name", ["cfg3", "cfg4"])
def test_full_size(H, name):
    """The n = 2^24 hull and the 10,000-cloud batch: every twin against the
    vectorised oracle (itself pinned to the definition on the CPU)."""
    import torch
    if name == "cfg3":
        p = workloads.cfg3()
        f = H.hull_sync(torch.from_numpy(p).cuda())
        fo = po = None
    else:
        from paper_1205_1171_amd import autotune
        pts, off, _ = workloads.cfg4()
        f, fo = H.hull_batched_sync(torch.from_numpy(pts).cuda(), off,
                                    schedule=autotune.lookup(off))
        po = torch.from_numpy(off).cuda()
    say("adjacency full size", name, f.shape[0])
    adj, open_edges = H.face_adjacency(f, fo, po)
    assert open_edges == 0
    ref = adjmod.adjacency_sorted(f.cpu().numpy(), None if fo is None else fo.cpu().numpy(),
                                  None if po is None else po.cpu().numpy())
    assert (adj.cpu().numpy() == ref).all()

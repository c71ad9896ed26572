"""Pins for the face-adjacency oracle: closed forms (tetrahedron, octahedron,
cube), the twin relation read back (an involution on half-edges), brute force
on small hulls, and the two oracle forms against each other."""
import numpy as np

import oracle
from oracle import adjacency as adjmod
from paper_1205_1171_amd import workloads


def brute(faces):
    f = np.asarray(faces).reshape(-1, 3)
    adj = np.full((len(f), 3), -1, dtype=np.int32)
    for r in range(len(f)):
        for k in range(3):
            a, b = f[r, k], f[r, (k + 1) % 3]
            for g in range(len(f)):
                for j in range(3):
                    if f[g, j] == b and f[g, (j + 1) % 3] == a:
                        adj[r, k] = g
    return adj


def test_tetrahedron_closed_form():
    faces = np.array([[0, 2, 1], [0, 1, 3], [1, 2, 3], [0, 3, 2]])
    adj = adjmod.adjacency(faces)
    for r in range(4):
        assert sorted(adj[r].tolist()) == sorted(set(range(4)) - {r})
    # the face across edge 0 -> 2 of face 0 holds 2 -> 0: face 3 (0, 3, 2)
    assert adj[0, 0] == 3


def test_octahedron_and_cube_from_oracle_hulls():
    for P in (workloads.octahedron(5), workloads.cube_corners(3)):
        faces = oracle.hull(P)
        adj = adjmod.adjacency(faces)
        assert (adj >= 0).all()
        assert (adj == brute(faces)).all()
        # every face has three distinct neighbours on these convex polytopes'
        # triangulations, none of them itself
        assert all(r not in adj[r] for r in range(len(faces)))


def _involution(faces, adj):
    f = np.asarray(faces).reshape(-1, 3)
    for r in range(len(f)):
        for k in range(3):
            g = adj[r, k]
            a, b = f[r, k], f[r, (k + 1) % 3]
            j = [jj for jj in range(3) if f[g, jj] == b and f[g, (jj + 1) % 3] == a]
            assert len(j) == 1 and adj[g, j[0]] == r


def test_random_hulls_brute_and_involution():
    rng = np.random.default_rng(3)
    for t in range(12):
        n = int(rng.integers(4, 60))
        P = workloads.lattice(rng, n, [1, 3, 100][t % 3])
        faces = oracle.hull(P)
        adj = adjmod.adjacency(faces)
        assert (adj == brute(faces)).all()
        assert (adj >= 0).all()
        _involution(faces, adj)


def test_sorted_form_matches_definition_in_batches():
    rng = np.random.default_rng(4)
    parts, offs = [], [0]
    for t in range(6):
        P = workloads.cube(rng, int(rng.integers(4, 300)), 1 << 20)
        f = oracle.hull(P)
        parts.append(f)
        offs.append(offs[-1] + len(f))
    faces = np.concatenate(parts)
    adj = adjmod.adjacency(faces, offs)
    assert (adj == adjmod.adjacency_sorted(faces, offs)).all()
    # an open surface: drop one face, its three neighbours lose a twin
    cut = np.delete(parts[0], 0, axis=0)
    a1 = adjmod.adjacency(cut)
    assert (a1 == -1).sum() == 3


def test_sorted_form_many_clouds():
    """More clouds than the (cloud, vertex) key holds: global vertex ids."""
    rng = np.random.default_rng(5)
    parts, offs, poffs = [], [0], [0]
    for t in range(1200):
        n = int(rng.integers(4, 9))
        f = oracle.hull(workloads.cube(rng, n, 1 << 10))
        parts.append(f)
        offs.append(offs[-1] + len(f))
        poffs.append(poffs[-1] + n)
    faces = np.concatenate(parts)
    adj = adjmod.adjacency(faces, offs)
    assert (adj == adjmod.adjacency_sorted(faces, offs, poffs)).all()

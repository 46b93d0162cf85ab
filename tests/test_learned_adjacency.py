"""Face adjacency of the leaves of a 2:1-balanced forest (host logic of the learned indicator's
evaluation: the variant of the combination in which the plain criterion decides on every leaf
next to one it refines)."""
import numpy as np
import torch

import oracle as orc
from paper_2406_11626_amd import scenarios
from paper_2406_11626_amd.learned import adjacent_fallback, face_neighbours


def _leaf(ids, t):
    return [p for p, r in enumerate(ids) if tuple(int(v) for v in r) == t][0]


def test_neighbours_across_same_coarser_and_finer_faces():
    m = orc.Mesh((3, 3, 3), (0.0, 0.0, 0.0), (3.0, 3.0, 3.0), 0, [(0, 1, 1, 1)])
    nb = face_neighbours(m.ids, (3, 3, 3))
    c = _leaf(m.ids, (0, 0, 1, 1))  # left of the refined centre cube
    got = {tuple(int(v) for v in m.ids[q]) for q in nb[c]}
    want = {(0, 0, 0, 1), (0, 0, 2, 1), (0, 0, 1, 0), (0, 0, 1, 2)}
    want |= {(1, 3, j, k) for j in range(3, 6) for k in range(3, 6)}  # the nine fine leaves across +x
    assert got == want
    f = _leaf(m.ids, (1, 3, 3, 3))  # the fine corner leaf: three coarser and three fine neighbours
    got = {tuple(int(v) for v in m.ids[q]) for q in nb[f]}
    assert got == {(0, 0, 1, 1), (0, 1, 0, 1), (0, 1, 1, 0), (1, 4, 3, 3), (1, 3, 4, 3), (1, 3, 3, 4)}


def test_periodic_wrap_and_symmetry_on_a_three_level_mesh():
    nb = face_neighbours(np.array([[0, 0, 0, 0], [0, 1, 0, 0]]), (2, 1, 1), periodic=True)
    assert [list(x) for x in nb] == [[1], [0]]  # x wraps onto the other leaf; y, z onto themselves
    w = scenarios.config(3)
    m = orc.Mesh(w.n0, w.origin, w.extent, w.bc, w.refined)
    nb = face_neighbours(m.ids, w.n0)
    for p, lst in enumerate(nb):
        assert p not in lst
        for q in lst:
            assert p in nb[q]  # sharing a face is symmetric
            assert abs(int(m.ids[p, 0]) - int(m.ids[q, 0])) <= 1
        # a leaf has at most 6 same-or-coarser neighbours and 9 finer ones per face
        assert len(lst) <= 54


def test_adjacent_fallback_drops_the_networks_additions_next_to_plain_refine():
    ids = np.array([[0, i, 0, 0] for i in range(5)])
    nb = face_neighbours(ids, (5, 1, 1))
    plain = torch.tensor([1, 0, 0, -1, 0], dtype=torch.int8)
    comb = torch.tensor([1, 1, 0, 1, 1], dtype=torch.int8)  # the network added leaves 1, 3, 4
    out = adjacent_fallback(comb, plain, nb)
    assert out.tolist() == [1, 0, 0, 1, 1]  # leaf 1 is next to the plain REFINE of leaf 0

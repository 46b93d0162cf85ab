"""Pins of the oracle's regrid (plan and state transfer): the refinement rules on hand-made tag
sets, the 2:1 face balance of every resulting mesh checked geometrically, and the transfer of
linear fields, which linear interpolation and cell averaging reproduce exactly."""
import numpy as np
import pytest

import oracle as orc
from seeded_inputs import box_centers


def leaf_boxes(m):
    """(n, 2, 3) lower and upper corners of each leaf's interior."""
    lo = m.geom[:, :3]
    return np.stack([lo, lo + 9 * m.geom[:, 3:]], axis=1)


def assert_face_balance(m):
    """Leaves that share a face area differ by at most one level (geometric check)."""
    b = leaf_boxes(m)
    lev = m.ids[:, 0]
    tol = 1e-9
    for p in range(m.np):
        for q in range(p + 1, m.np):
            touch, overlap = 0, 0
            for a in range(3):
                if abs(b[p, 1, a] - b[q, 0, a]) < tol or abs(b[q, 1, a] - b[p, 0, a]) < tol:
                    touch += 1
                elif min(b[p, 1, a], b[q, 1, a]) - max(b[p, 0, a], b[q, 0, a]) > tol:
                    overlap += 1
            if touch == 1 and overlap == 2:
                assert abs(int(lev[p]) - int(lev[q])) <= 1, (m.ids[p], m.ids[q])


def as_set(cubes):
    return {tuple(int(v) for v in c) for c in cubes}


BC_SOMMERFELD, NV = 2, 59


def mesh(refined, n0=(4, 4, 4), bc=BC_SOMMERFELD):
    return orc.Mesh(n0, (0.0, 0.0, 0.0), (4.0, 4.0, 4.0), bc, refined)


def leaf_index(m, lev, i, j, k):
    hit = np.where((m.ids == np.array([lev, i, j, k])).all(axis=1))[0]
    return int(hit[0]) if hit.size else -1


def test_keep_tags_leave_the_mesh_unchanged():
    m = mesh([(0, 1, 1, 1), (1, 4, 4, 4)])
    assert as_set(m.regrid_plan(np.zeros(m.np, np.int8), 3)) == {(0, 1, 1, 1), (1, 4, 4, 4)}


def test_refinement_is_balanced_by_refining_coarse_neighbours():
    m = mesh([(0, 1, 1, 1)])
    tags = np.zeros(m.np, np.int8)
    tags[leaf_index(m, 1, 3, 3, 3)] = 1  # the corner child of cube (1,1,1) touching x = y = z = 1
    plan = as_set(m.regrid_plan(tags, 2))
    assert (1, 3, 3, 3) in plan and (0, 1, 1, 1) in plan
    # its level-2 children face the level-0 leaves across x, y and z = 1: those are refined
    assert {(0, 0, 1, 1), (0, 1, 0, 1), (0, 1, 1, 0)} <= plan
    n = mesh(sorted(plan))
    assert_face_balance(n)
    # max_level stops the refinement of level-1 leaves
    assert as_set(m.regrid_plan(tags, 1)) == {(0, 1, 1, 1)}


def test_coarsening_of_whole_families_only():
    m = mesh([(0, 1, 1, 1), (0, 2, 1, 1)])
    fam = [leaf_index(m, 1, 3 + u, 3 + v, 3 + w) for w in range(3) for v in range(3) for u in range(3)]
    tags = np.zeros(m.np, np.int8)
    tags[fam] = -1
    assert as_set(m.regrid_plan(tags, 2)) == {(0, 2, 1, 1)}
    tags[fam[13]] = 0
    assert as_set(m.regrid_plan(tags, 2)) == {(0, 1, 1, 1), (0, 2, 1, 1)}
    # a refined level-1 neighbour across the family's face blocks the merge
    m2 = mesh([(0, 1, 1, 1), (0, 2, 1, 1), (1, 6, 4, 4)])
    t2 = np.zeros(m2.np, np.int8)
    t2[[leaf_index(m2, 1, 3 + u, 3 + v, 3 + w) for w in range(3) for v in range(3) for u in range(3)]] = -1
    assert as_set(m2.regrid_plan(t2, 3)) == {(0, 1, 1, 1), (0, 2, 1, 1), (1, 6, 4, 4)}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_tags_give_balanced_meshes(seed):
    rng = np.random.default_rng(seed)
    m = mesh([(0, 1, 1, 1), (0, 2, 2, 1), (1, 4, 4, 4)])
    tags = rng.choice(np.array([-1, 0, 0, 1], np.int8), m.np)
    plan = m.regrid_plan(tags, 3)
    n = mesh([tuple(c) for c in plan])
    assert_face_balance(n)
    for p in np.where(tags == 1)[0]:
        lev, i, j, k = m.ids[p]
        if lev < 3:
            assert leaf_index(n, lev, i, j, k) < 0  # a tagged leaf is no longer a leaf


def linear_state(m, coef):
    """Every slot v is coef[v, 0] + coef[v, 1:] . x at the cell centres (whole boxes)."""
    Q = m.zeros()
    for p in range(m.np):
        P = box_centers(m.geom[p, :3], m.geom[p, 3:])
        Q[p] = coef[:, 0] + P @ coef[:, 1:].T
    return Q


def test_transfer_reproduces_linear_fields():
    rng = np.random.default_rng(5)
    coef = rng.normal(size=(NV, 4))
    m = mesh([(0, 1, 1, 1), (0, 2, 1, 1)])
    tags = np.zeros(m.np, np.int8)
    tags[[leaf_index(m, 1, 3 + u, 3 + v, 3 + w) for w in range(3) for v in range(3) for u in range(3)]] = -1
    tags[leaf_index(m, 0, 3, 3, 3)] = 1
    tags[leaf_index(m, 1, 7, 4, 4)] = 1
    n = mesh([tuple(c) for c in m.regrid_plan(tags, 2)])
    kinds = {"copy": 0, "prolong": 0, "restrict": 0}
    for lev, i, j, k in n.ids:
        if leaf_index(m, lev, i, j, k) >= 0:
            kinds["copy"] += 1
        elif lev > 0 and leaf_index(m, lev - 1, i // 3, j // 3, k // 3) >= 0:
            kinds["prolong"] += 1
        else:
            kinds["restrict"] += 1
    assert min(kinds.values()) > 0, kinds
    Qo = linear_state(m, coef)
    Qn = n.zeros()
    m.regrid_transfer(Qo, n, Qn)
    want = linear_state(n, coef)
    inner = (slice(None), slice(3, 12), slice(3, 12), slice(3, 12))
    assert np.allclose(Qn[inner], want[inner], rtol=0, atol=1e-12 * np.abs(want).max())

"""The oracle's coarse-fine halo fill against the transfer matrices printed in App. E
(tests/golden/app_e_transfer_matrices.txt), which act on a whole coarse face of 9 x 9 volumes
and the 27 x 27 fine volumes behind it.  On the two-level mesh, random values in a coarse leaf's
interior (fine interiors zero) must reach a fine neighbour's ghost layers exactly through
P_par x P_par x P_perp, and random values in a fine leaf's interior (everything else zero) must
reach the coarse neighbour's halo exactly through R_par x R_par x R_perp.  Three faces with
different normals, sides and offsets within the coarse face check the axis and orientation
bookkeeping, and the fine leaves at the edge of a coarse face check the extrapolating rows."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as orc

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "app_e_transfer_matrices.txt")


def load_matrices():
    mats, cur = {}, None
    with open(GOLDEN) as fh:
        lines = fh.read().splitlines()
    for ln in lines:
        ln = ln.strip()
        if not ln or ln.startswith("#"):
            continue
        if ln.startswith("["):
            cur = ln[1:-1]
            mats[cur] = []
        else:
            mats[cur].append([float(Fraction(t)) for t in ln.split()])
    return {k: np.array(v) for k, v in mats.items()}


M = load_matrices()


def test_golden_matrices_shapes_and_consistency():
    assert M["P_par"].shape == (27, 9) and M["P_perp"].shape == (3, 6)
    assert M["R_par"].shape == (9, 27) and M["R_perp"].shape == (3, 6)
    for k in M:  # every operator reproduces constants
        np.testing.assert_allclose(M[k].sum(axis=1), 1.0, atol=1e-15)


def mesh():
    """3^3 level-0 cubes on [0,3]^3 with the centre cube refined (27 level-1 leaves)."""
    return orc.Mesh([3, 3, 3], [0, 0, 0], [3.0, 3.0, 3.0], bc=0, refined=[(0, 1, 1, 1)])


def leaf(m, ids):
    return [p for p in range(m.np) if tuple(m.ids[p]) == tuple(ids)][0]


def take(box, a, sel, tang):
    """Layer sel along axis a of a leaf's (z, y, x, slot) box, restricted to tang[0], tang[1]
    along the two other axes taken in increasing order; dims (tangential 0, tangential 1, slot)."""
    idx = [None] * 3
    others = [b for b in range(3) if b != a]
    idx[2 - a] = sel
    idx[2 - others[0]] = tang[0]
    idx[2 - others[1]] = tang[1]
    # the box stores the higher axis first, so the remaining dims are (others[1], others[0])
    return box[tuple(idx)].swapaxes(0, 1)


# (fine leaf (level, i, j, k), normal axis, side of the fine leaf's face)
FACES = [((1, 3, 3, 5), 0, -1), ((1, 5, 5, 3), 1, +1), ((1, 4, 3, 3), 2, -1)]


def geometry(fine, a, s):
    f = np.array(fine[1:])
    c = f // 3
    c[a] = (f[a] + s) // 3
    others = [b for b in range(3) if b != a]
    off = [int(f[b] - 3 * c[b]) for b in others]  # fine leaf's third of the coarse face
    coarse = (0, *c.tolist())
    # layer -> box index along a, in the enumeration of the golden file
    f_ghost = [k if s < 0 else 14 - k for k in range(3)]
    f_inner = [3 + q if s < 0 else 11 - q for q in range(3)]
    c_inner = [9 + n if s < 0 else 5 - n for n in range(3)]
    c_halo = [12 + n if s < 0 else 2 - n for n in range(3)]
    win = [slice(3 + 3 * o, 6 + 3 * o) for o in off]
    fine_rows = [slice(9 * o, 9 * o + 9) for o in off]  # the fine leaf's rows of P_par
    return coarse, f_ghost, f_inner, c_inner, c_halo, win, fine_rows


@pytest.mark.parametrize("fine,a,s", FACES)
def test_prolongation_is_the_printed_P(fine, a, s):
    m = mesh()
    coarse, f_ghost, _, c_inner, _, _, rows = geometry(fine, a, s)
    pf, pc = leaf(m, fine), leaf(m, coarse)
    rng = np.random.default_rng(11)
    Q = m.zeros()
    Q[pc, 3:12, 3:12, 3:12] = rng.normal(size=(9, 9, 9, 59))
    m.fill_halos(Q)
    face = (slice(3, 12), slice(3, 12))
    C = np.stack([take(Q[pc], a, c_inner[n], face) for n in range(3)])  # (n, l, m, slot)
    Pperp = M["P_perp"][:, :3]  # the restricted layers c3..c5 are zero here
    want = np.einsum("kn,il,jm,nlms->kijs", Pperp, M["P_par"][rows[0]], M["P_par"][rows[1]], C)
    got = np.stack([take(Q[pf], a, f_ghost[k], (slice(3, 12), slice(3, 12))) for k in range(3)])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)
    assert np.abs(want).max() > 0.5


@pytest.mark.parametrize("fine,a,s", FACES)
def test_restriction_is_the_printed_R(fine, a, s):
    m = mesh()
    coarse, _, f_inner, _, c_halo, win, rows = geometry(fine, a, s)
    pf, pc = leaf(m, fine), leaf(m, coarse)
    rng = np.random.default_rng(12)
    Q = m.zeros()
    Q[pf, 3:12, 3:12, 3:12] = rng.normal(size=(9, 9, 9, 59))
    m.fill_halos(Q)
    F = np.stack([take(Q[pf], a, f_inner[q], (slice(3, 12), slice(3, 12))) for q in range(3)])
    Rperp = M["R_perp"][:, 3:]  # columns f3..f5; the ghost columns f0..f2 are zero
    assert np.all(M["R_perp"][:, :3] == 0)
    want = np.einsum("nq,li,mj,qijs->nlms", Rperp, M["R_par"][win[0].start - 3:win[0].stop - 3, rows[0]],
                     M["R_par"][win[1].start - 3:win[1].stop - 3, rows[1]], F)
    got = np.stack([take(Q[pc], a, c_halo[n], win) for n in range(3)])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)
    assert np.abs(want).max() > 0.5

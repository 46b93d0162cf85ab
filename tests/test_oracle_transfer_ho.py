"""Pins of the oracle's higher-order coarse-fine operators (transfer = 1; the paper names
higher-order interpolation and restriction as the remedy for reflections at refinement
boundaries): quadratic fields are reproduced exactly on every coarse-fine halo, the restricted
coarse halo cells are the fine cells with the same centre, and a cubic along the normal leaves
exactly the three-point Lagrange remainder in the prolonged fine ghosts."""
import numpy as np

import oracle as orc
from gpu_helpers import SLABS


def amr_mesh():
    m = orc.Mesh([3, 3, 3], [0, 0, 0], [3.0, 3.0, 3.0], bc=0, refined=[(0, 1, 1, 1)])
    m.set_transfer(1)
    return m


def coarse_fine_halos(m):
    """(leaf, index) of the halo slabs of faces between the refined centre cube and its six
    coarse neighbours, on both sides."""
    out = []
    for p in range(m.np):
        lev, i, j, k = m.ids[p]
        if lev == 0 and abs(i - 1) + abs(j - 1) + abs(k - 1) != 1:
            continue
        X = m.cell_centers(p)
        for a in range(3):
            for side in (0, 1):
                idx = [slice(3, 12)] * 3
                idx[2 - a] = slice(0, 3) if side == 0 else slice(12, 15)
                cc = X[tuple(idx)]
                if np.any(cc < 0) or np.any(cc > 3):
                    continue
                inner = (cc >= 1) & (cc <= 2)
                if lev == 0 and not np.all(inner):
                    continue
                if lev == 1 and np.all(inner):
                    continue
                out.append((p, tuple(idx)))
    return out


def test_quadratic_fields_reproduced_on_every_coarse_fine_halo():
    m = amr_mesh()
    rng = np.random.default_rng(0)
    b = rng.normal(size=3)
    C = rng.normal(size=(3, 3))
    C = C + C.T

    def f(X):
        Y = X - 1.5
        return 0.4 + Y @ b + np.einsum("...i,ij,...j->...", Y, C, Y)

    Q = m.zeros()
    for p in range(m.np):
        Q[p] = f(m.cell_centers(p))[..., None] * np.linspace(1, 2, 59)
    exact = Q.copy()
    Q[:, SLABS] = np.nan
    m.fill_halos(Q)
    halos = coarse_fine_halos(m)
    assert len(halos) == 6 + 6 * 9
    for p, idx in halos:
        assert np.all(np.isfinite(Q[p][idx]))
        np.testing.assert_allclose(Q[p][idx], exact[p][idx], rtol=0, atol=1e-12 * np.abs(exact).max())


def test_restricted_halos_are_the_coincident_fine_cells():
    m = amr_mesh()
    rng = np.random.default_rng(1)
    Q = rng.normal(size=m.zeros().shape)
    m.fill_halos(Q)
    fine = [p for p in range(m.np) if m.ids[p, 0] == 1]
    centres = {}
    for p in fine:
        X = m.cell_centers(p)
        for z in range(3, 12):
            for y in range(3, 12):
                for x in range(3, 12):
                    centres[tuple(np.round(X[z, y, x] * 54).astype(int))] = Q[p, z, y, x]
    n = 0
    for p, idx in coarse_fine_halos(m):
        if m.ids[p, 0] != 0:
            continue
        X = m.cell_centers(p)[idx]
        V = Q[p][idx]
        for key, v in zip(np.round(X.reshape(-1, 3) * 54).astype(int), V.reshape(-1, 59)):
            assert np.array_equal(centres[tuple(key)], v)
            n += 1
    assert n == 6 * 3 * 81


def test_cubic_normal_remainder_in_prolonged_ghosts():
    """f = (x - 1)^3 near the -x face of the refined cube: the fine ghost L sits at s = 1/2 -
    (L - 1/2)/3 coarse cells from the centre of c2 towards the face, c1, c2 and the injected c3
    are exact, so the ghost holds f + H^3 s (1 - s^2) with H = 1/9 (the Lagrange remainder)."""
    m = amr_mesh()
    Q = m.zeros()
    for p in range(m.np):
        X = m.cell_centers(p)
        Q[p] = ((X[..., 0] - 1.0) ** 3)[..., None]
    m.fill_halos(Q)
    H = 1.0 / 9
    p = [q for q in range(m.np) if tuple(m.ids[q]) == (1, 3, 4, 4)][0]
    X = m.cell_centers(p)
    for L in (1, 2, 3):
        s = 0.5 - (L - 0.5) / 3.0
        col = 3 - L  # box x index of ghost layer L on the -x side
        got = Q[p, 3:12, 3:12, col, 0]
        want = (X[3:12, 3:12, col, 0] - 1.0) ** 3 + H ** 3 * s * (1 - s * s)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)

"""Pins of the oracle's mesh-level operations (no GPU): halo filling and the App. E transfer
operators, the RK4 stage combine, the algebraic projection, the constraint monitor, the
Sommerfeld ghosts and the gauge-wave evolution against the exact solution."""
import math

import numpy as np
import pytest

import exact_ccz4 as ex
import oracle as orc
from seeded_inputs import box_points, smooth_state

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def face_slab_mask():
    """Boolean (15,15,15) mask of the six face halo slabs (no edges, no corners)."""
    m = np.zeros((15, 15, 15), bool)
    inner = slice(3, 12)
    for a in range(3):
        for sl in (slice(0, 3), slice(12, 15)):
            idx = [inner, inner, inner]
            idx[2 - a] = sl
            m[tuple(idx)] = True
    return m


SLABS = face_slab_mask()


# ------------------------------------------------------------------ uniform grids

def test_periodic_fill_equals_global_window():
    """On a uniform periodic grid every face halo equals the window of one global array
    (wrapped), bit for bit."""
    m = orc.Mesh([3, 2, 4], [0, 0, 0], [3.0, 2.0, 4.0], bc=0)
    rng = np.random.default_rng(0)
    G = rng.normal(size=(36, 18, 27, 59))  # [z, y, x, slot] of the level-0 cells
    Q = m.zeros()
    for p, (lev, i, j, k) in enumerate(m.ids):
        Q[p, 3:12, 3:12, 3:12] = G[9 * k:9 * k + 9, 9 * j:9 * j + 9, 9 * i:9 * i + 9]
    Q[:, SLABS] = np.nan
    m.fill_halos(Q)
    for p, (lev, i, j, k) in enumerate(m.ids):
        zs = (np.arange(15) - 3 + 9 * k) % 36
        ys = (np.arange(15) - 3 + 9 * j) % 18
        xs = (np.arange(15) - 3 + 9 * i) % 27
        W = G[np.ix_(zs, ys, xs)]
        assert np.array_equal(Q[p][SLABS], W[SLABS])


def test_neumann_fill_copies_boundary_layer():
    m = orc.Mesh([2, 1, 1], [0, 0, 0], [2.0, 1.0, 1.0], bc=1)
    rng = np.random.default_rng(1)
    Q = rng.normal(size=(2, 15, 15, 15, 59))
    m.fill_halos(Q)
    # patch 0: -x face is physical, +x face copies patch 1
    for L in range(3):
        assert np.array_equal(Q[0, 3:12, 3:12, L], Q[0, 3:12, 3:12, 3])
        assert np.array_equal(Q[0, 3:12, 3:12, 12 + L], Q[1, 3:12, 3:12, 3 + L])
        assert np.array_equal(Q[1, 3:12, 3:12, 12 + L], Q[1, 3:12, 3:12, 11])
        assert np.array_equal(Q[0, 3:12, L, 3:12], Q[0, 3:12, 3, 3:12])
        assert np.array_equal(Q[0, 14 - L, 3:12, 3:12], Q[0, 11, 3:12, 3:12])


# ------------------------------------------------------------------ AMR transfer (App. E)

def amr_mesh(bc=0):
    """3^3 level-0 cubes on [0,3]^3 with the centre cube refined (27 level-1 leaves)."""
    return orc.Mesh([3, 3, 3], [0, 0, 0], [3.0, 3.0, 3.0], bc=bc, refined=[(0, 1, 1, 1)])


def _fill_linear(m, coef):
    Q = m.zeros()
    for p in range(m.np):
        X = m.cell_centers(p)
        val = coef[0] + X @ coef[1:4]
        Q[p] = val[..., None] * np.linspace(1, 2, 59)
    return Q


def test_amr_mesh_leaves_and_geometry():
    m = amr_mesh()
    assert m.np == 26 + 27
    assert (m.ids[:, 0] == 0).sum() == 26 and (m.ids[:, 0] == 1).sum() == 27
    # canonical order: level, then k, j, i
    keys = [(l, k, j, i) for (l, i, j, k) in m.ids]
    assert keys == sorted(keys)
    fine = m.geom[m.ids[:, 0] == 1]
    assert np.allclose(fine[:, 3:], 1.0 / 27)


def test_transfer_operators_exact_for_linear_fields_and_ordering():
    """Restriction (R_avg x R_avg x R_perp) and prolongation (P_par x P_par x P_perp) reproduce
    linear fields exactly on every coarse-fine face.  Halos start as NaN: the prolongation
    reads the restricted layer c3, so an exact, finite result also shows restriction ran
    first."""
    m = amr_mesh()
    coef = np.array([0.3, 1.1, -0.7, 0.45])
    Q = _fill_linear(m, coef)
    Qexact = Q.copy()
    Q[:, SLABS] = np.nan
    m.fill_halos(Q)
    for p in range(m.np):
        lev, i, j, k = m.ids[p]
        X = m.cell_centers(p)
        if lev == 1 or (abs(i - 1) + abs(j - 1) + abs(k - 1) == 1):
            for a in range(3):
                for side in (0, 1):
                    idx = [slice(3, 12)] * 3
                    idx[2 - a] = slice(0, 3) if side == 0 else slice(12, 15)
                    got = Q[p][tuple(idx)]
                    # periodic images are not linear: skip faces on the domain boundary
                    cc = X[tuple(idx)]
                    if np.any(cc < 0) or np.any(cc > 3):
                        continue
                    assert np.all(np.isfinite(got))
                    np.testing.assert_allclose(got, Qexact[p][tuple(idx)], rtol=0, atol=1e-12)


def test_transfer_rows_sum_to_one_and_restriction_preserves_mean():
    """A constant field is reproduced by both operators; the averaging restriction of a field
    that varies only tangentially keeps the face mean."""
    m = amr_mesh()
    Q = m.zeros() + 2.5
    Q[:, SLABS] = np.nan
    m.fill_halos(Q)
    assert np.all(np.abs(Q[:, SLABS] - 2.5) < 1e-13)
    # tangential-only field on the fine side of the -x face of the coarse cube (2,1,1):
    # c3 (R_perp row 1 = average of f3..f5) keeps the mean of the 27x27 fine face.
    Q = m.zeros()
    rng = np.random.default_rng(3)
    for p in range(m.np):
        if m.ids[p, 0] == 1:
            Q[p, 3:12, 3:12, 3:12] = rng.normal(size=(9, 9, 1, 59))
    m.fill_halos(Q)
    pc = [p for p in range(m.np) if tuple(m.ids[p]) == (0, 2, 1, 1)][0]
    kids = [p for p in range(m.np) if m.ids[p, 0] == 1 and m.ids[p, 1] == 5]
    fine_mean = np.mean([Q[p, 3:12, 3:12, 11] for p in kids], axis=(0, 1, 2))
    coarse_mean = Q[pc, 3:12, 3:12, 2].mean(axis=(0, 1))
    np.testing.assert_allclose(coarse_mean, fine_mean, atol=1e-13)


def test_prolongation_quadratic_error_closed_form():
    """For f = x^2 along the face normal the prolonged fine ghost layers carry the linear-
    interpolation error: ghost f0 at -2.5h reads c1/3 + 2c2/3, error (1/3)(2/3) H^2 with H = 3h,
    i.e. 2 h^2 for the coarse-cell spacing H (and 0 at f1 = c2)."""
    m = amr_mesh()
    Q = m.zeros()
    for p in range(m.np):
        X = m.cell_centers(p)
        Q[p] = ((X[..., 0] - 1.0) ** 2)[..., None]
    m.fill_halos(Q)
    h = 1.0 / 27
    # fine leaf (1, 3, 4, 4): its -x face borders the coarse cube (0,0,1,1)
    p = [p for p in range(m.np) if tuple(m.ids[p]) == (1, 3, 4, 4)][0]
    X = m.cell_centers(p)
    err = Q[p, 3:12, 3:12, 0:3, 0] - (X[3:12, 3:12, 0:3, 0] - 1.0) ** 2
    np.testing.assert_allclose(err[..., 0], 2 * h * h, atol=1e-12)   # f0
    np.testing.assert_allclose(err[..., 1], 0.0, atol=1e-12)          # f1 = c2
    # f2 = 2/3 c2 + 1/3 c3, where c3 is the restricted (exact average of f3..f5 + O(h^2))


# ------------------------------------------------------------------ RK4 and projection

def test_rk4_stages_reproduce_taylor_polynomial():
    """With k_s = lam * Q_s per slot, the four stage combines give
    Q^{n+1} = sum_{m<=4} (lam dt)^m / m! Q^n (classical RK4 on a linear ODE)."""
    m = orc.Mesh([1, 1, 1], [0, 0, 0], [1.0, 1.0, 1.0], bc=0)
    rng = np.random.default_rng(4)
    Qn = m.zeros()
    Qn[..., :] = rng.normal(size=59)
    Qn[..., 0:6] = [1, 0, 0, 1, 0, 1]
    Qn[..., 11:17] = 0.0
    lam = rng.normal(size=59)
    lam[0:6] = 0.0
    lam[11:17] = 0.0
    dt = 0.1
    acc, Qs = m.zeros(), Qn.copy()
    Qnew = m.zeros()
    for s in range(4):
        k = lam * Qs
        Qnext = Qnew if s == 3 else m.zeros()
        m.rk4_stage(s, dt, Qn, k, acc, Qnext)
        Qs = Qnext
    z = lam * dt
    exp = Qn * (1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24)
    I = slice(3, 12)
    np.testing.assert_allclose(Qnew[:, I, I, I], exp[:, I, I, I], rtol=1e-14, atol=1e-14)
    with pytest.raises(ValueError):
        m.rk4_stage(4, dt, Qn, Qn, acc, Qnew)
    with pytest.raises(ValueError):
        m.rk4_stage(0, -1.0, Qn, Qn, acc, Qnew)


def test_projection_enforces_algebraic_constraints():
    rng = np.random.default_rng(5)
    for seed in range(5):
        q = smooth_state(rng.uniform(-1, 1, (1, 3)), seed)[0]
        p = orc.project_point(q)
        g = np.array([[p[SYM.index((min(i, j), max(i, j)))] for j in range(3)] for i in range(3)])
        A = np.array([[p[11 + SYM.index((min(i, j), max(i, j)))] for j in range(3)] for i in range(3)])
        assert abs(np.linalg.det(g) - 1) < 1e-14
        assert abs(np.sum(np.linalg.inv(g) * A)) < 1e-14
        g0 = np.array([[q[SYM.index((min(i, j), max(i, j)))] for j in range(3)] for i in range(3)])
        np.testing.assert_allclose(g, g0 / np.linalg.det(g0) ** (1 / 3), rtol=1e-14)
        np.testing.assert_allclose(orc.project_point(p), p, atol=1e-15)
        others = [v for v in range(59) if v not in range(0, 6) and v not in range(11, 17)]
        assert np.array_equal(p[others], q[others])
    q = orc.init_point(0, [0.1, 2.0], [0.123, 0.4, -0.2])
    np.testing.assert_allclose(orc.project_point(q), q, atol=1e-15)


# ------------------------------------------------------------------ constraints

def _cons_err(Qf, center, h, hm_exact=None):
    pts = box_points(center, h)
    Q = ex.evaluate(Qf, pts)
    hm = orc.constraints_box([h, h, h], Q)
    ref = np.zeros_like(hm) if hm_exact is None else hm_exact(pts[3:12, 3:12, 3:12].reshape(-1, 3))
    return np.abs(hm - ref).max(0)


@pytest.mark.parametrize("name", ["puncture", "distorted_minkowski", "gauge_wave"])
def test_constraints_vanish_on_exact_data(name):
    Qf = {
        "puncture": ex.ccz4_from_adm(ex.adm_puncture(1.0)),
        "distorted_minkowski": ex.ccz4_from_adm(ex.adm_from_g4(ex.g4_distorted_minkowski(0.05))),
        "gauge_wave": ex.ccz4_from_adm(ex.adm_from_g4(ex.g4_gauge_wave(0.1, 2.0, (1, 2, 3)))),
    }[name]
    center = (1.7, -1.1, 0.9) if name == "puncture" else (0.13, 0.21, -0.17)
    e1 = _cons_err(Qf, center, 0.04)
    e2 = _cons_err(Qf, center, 0.02)
    assert e1.max() / e2.max() > 12.0
    assert e2.max() < 1e-5


def test_constraints_brill_lindquist_bowen_york_closed_form():
    """Brill-Lindquist conformal factor with Bowen-York curvature and no puncture correction:
    R = 0 (psi harmonic), so H = -psi^-12 sum Ahat_ij^2 and M_i = 0 (Ahat is divergence free)."""
    import torch
    holes = [(0.5, (3.0, 0.0, 0.0), (0.0, 0.095, 0.0)), (0.5, (-3.0, 0.0, 0.0), (0.0, -0.095, 0.0))]
    Qf = ex.ccz4_from_adm(ex.adm_brill_lindquist_bowen_york(holes))

    def hm_exact(pts):
        out = np.zeros((pts.shape[0], 4))
        for n, p in enumerate(pts):
            X = torch.tensor([0.0, *p])
            Ah = ex.bowen_york_Ahat(X, holes)
            psi = ex.brill_lindquist_psi(X, holes)
            out[n, 0] = float(-psi ** -12 * torch.sum(Ah * Ah))
        return out

    c = (1.2, 0.8, -0.6)
    e1 = _cons_err(Qf, c, 0.08, hm_exact)
    e2 = _cons_err(Qf, c, 0.04, hm_exact)
    assert e1.max() / e2.max() > 12.0
    assert e2.max() < 1e-6


def test_constraint_norms_and_nonfinite_count():
    m = orc.Mesh([2, 2, 2], [-9, -9, -9], [18.0, 18.0, 18.0], bc=1)
    Q = m.zeros()
    m.init(Q, 1, [1.0, 0.0, 0.0, 0.0, 0])
    m.fill_halos(Q)
    norms, HM = m.constraints(Q, want_fields=True)
    assert norms[2] == 0
    np.testing.assert_allclose(norms[0], np.sqrt(np.mean(HM[..., 0] ** 2)), rtol=1e-14)
    np.testing.assert_allclose(norms[1], np.sqrt(np.mean(np.sum(HM[..., 1:] ** 2, -1))), rtol=1e-14)
    Q[1, 5, 6, 7, 17] = np.nan
    norms2 = m.constraints(Q)
    assert norms2[2] >= 1


# ------------------------------------------------------------------ Sommerfeld ghosts

def test_sommerfeld_ghosts_approximate_outgoing_wave():
    """For Q = Q_ini + u(r - t)/r the ghost right-hand side G_L (layered radiative condition)
    approaches the exact d_t Q = -u'(r - t)/r at first order in dx."""
    errs = []
    for n in (1, 2):
        m = orc.Mesh([2 * n, 2 * n, 2 * n], [-4, -4, -4], [8.0, 8.0, 8.0], bc=2)
        Q0 = m.zeros()
        Q0[..., [0, 3, 5, 6, 10]] = 1.0
        m.set_background(Q0)
        Q = Q0.copy()
        dtQ = m.zeros()
        u = lambda s: 0.01 * np.exp(-((s - 5.0) ** 2) / 2)
        up = lambda s: -(s - 5.0) * u(s)
        for p in range(m.np):
            X = m.cell_centers(p)
            r = np.linalg.norm(X, axis=-1)
            Q[p] += (u(r) / r)[..., None]
            dtQ[p] = (-up(r) / r)[..., None]
        k = m.rhs(orc.params(), Q)
        err = 0.0
        for p in range(m.np):
            e = np.abs(k[p][SLABS] - dtQ[p][SLABS])[:, :58]
            touched = np.abs(k[p][SLABS][:, :58]).max(axis=1) > 0
            if touched.any():
                err = max(err, e[touched].max())
        errs.append(err)
    assert errs[0] / errs[1] > 1.6, errs
    assert errs[1] < 5e-4


# ------------------------------------------------------------------ evolution

@pytest.mark.slow
def test_gauge_wave_rk4_converges_to_exact_solution():
    """The paper's first benchmark reduced to a thin periodic slab (the wave depends on x only):
    FD4 + KO 0.1 + RK4 at CFL 0.1 against the exact gauge wave at t = T converges at fourth
    order, the order the paper reports for RK4 with a small KO coefficient."""
    A, k = 0.1, 2.0
    Qf = ex.ccz4_from_adm(ex.adm_from_g4(ex.g4_gauge_wave(A, k, (1, 0, 0))))
    pr = orc.params(kappa1=1.0, kappa2=0.0, kappa3=0.0, ko_eps=0.1, slicing=0, shift=0)
    T = 8 * 0.1 / 27
    errs = []
    for npx in (3, 6):
        h = 1.0 / (9 * npx)
        m = orc.Mesh([npx, 1, 1], [-0.5, 0, 0], [1.0, 9 * h, 9 * h], bc=0)
        Q = m.zeros()
        m.init(Q, 0, [A, k])
        nsteps = int(round(T / (0.1 * h)))
        for _ in range(nsteps):
            Q = m.rk4_step(pr, Q, 0.1 * h)
        err = 0.0
        for p in range(m.np):
            X = m.cell_centers(p)[3:12, 3:12, 3:12]
            Qx = ex.evaluate(Qf, X, t=T)
            err = max(err, np.abs(Q[p, 3:12, 3:12, 3:12] - Qx).max())
        errs.append(err)
    assert errs[0] / errs[1] > 12.0, errs
    assert errs[1] < 1e-5

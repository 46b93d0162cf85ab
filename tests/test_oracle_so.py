"""Pins of the oracle's second-order formulation (Sec. 2.2; Sec. 3.2 "explicit gradient reconstruction";
Algorithm 2, and the remark of App. B that the red terms belong to the first-order system only):
the reconstruction of A, B, D, P is exact on quartic primaries, the right-hand side of the
primaries still converges to the exact time derivative at fourth order, and a trace shift of
At changes it by a closed form that differs from the first-order one by exactly the red terms'
share."""
import numpy as np
import pytest

import exact_ccz4 as ex
import oracle as orc
from seeded_inputs import box_centers, box_points, smooth_state

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def s_sym(i, j):
    return {(0, 0): 0, (0, 1): 1, (0, 2): 2, (1, 1): 3, (1, 2): 4, (2, 2): 5}[(min(i, j), max(i, j))]


def quartic(P, c):
    """sum_e c_e x^a y^b z^c over the monomials of degree <= 4, and its gradient."""
    x, y, z = P[..., 0], P[..., 1], P[..., 2]
    v = np.zeros(P.shape[:-1])
    g = np.zeros(P.shape)
    n = 0
    for a in range(5):
        for b in range(5 - a):
            for cc in range(5 - a - b):
                w = c[n]
                n += 1
                v += w * x ** a * y ** b * z ** cc
                if a:
                    g[..., 0] += w * a * x ** (a - 1) * y ** b * z ** cc
                if b:
                    g[..., 1] += w * b * x ** a * y ** (b - 1) * z ** cc
                if cc:
                    g[..., 2] += w * cc * x ** a * y ** b * z ** (cc - 1)
    return v, g


def test_reconstruction_exact_on_quartic_primaries():
    """FD4 is exact on polynomials of degree 4, so A_k = d_k alpha, B_k^i = d_k beta^i,
    D_kij = d_k gt_ij / 2 and P_k = d_k phi come out exact (to rounding) on a patch whose 11
    primaries are random quartics; the primaries themselves are left untouched."""
    rng = np.random.default_rng(7)
    m = orc.Mesh((1, 1, 1), (0.2, -0.1, 0.3), (0.45, 0.45, 0.45), 1)
    P = box_centers(m.geom[0, :3], m.geom[0, 3:])
    Q = m.zeros()
    grads = {}
    for v in range(11):
        val, g = quartic(P, rng.normal(size=35))
        Q[0, ..., v] = val
        grads[v] = g
    Q[0, ..., 11:] = rng.normal(size=Q[0, ..., 11:].shape)
    before = Q.copy()
    m.reconstruct(Q)
    I = (0, slice(3, 12), slice(3, 12), slice(3, 12))
    scale = max(np.abs(g[3:12, 3:12, 3:12]).max() for g in grads.values())
    tol = 1e-11 * scale
    for k in range(3):
        np.testing.assert_allclose(Q[I + (25 + k,)], grads[6][3:12, 3:12, 3:12, k], rtol=0, atol=tol)
        np.testing.assert_allclose(Q[I + (55 + k,)], grads[10][3:12, 3:12, 3:12, k], rtol=0, atol=tol)
        for i in range(3):
            np.testing.assert_allclose(Q[I + (28 + 3 * k + i,)], grads[7 + i][3:12, 3:12, 3:12, k], rtol=0, atol=tol)
        for n_ in range(6):
            np.testing.assert_allclose(Q[I + (37 + 6 * k + n_,)], 0.5 * grads[n_][3:12, 3:12, 3:12, k], rtol=0,
                                       atol=tol)
    # everything but the interior auxiliaries is as before
    changed = np.zeros(Q.shape, bool)
    changed[I + (slice(25, 58),)] = True
    assert np.array_equal(Q[~changed], before[~changed])


def _generic_point(seed):
    rng = np.random.default_rng(seed)
    q = smooth_state(rng.uniform(-1, 1, (1, 3)), seed)[0]
    dq = rng.normal(size=(3, 59)) * 0.2
    return q, dq


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_trace_shift_closed_form_without_red_terms(seed):
    """Shift At -> At + lam gt with d_k At shifted consistently (d_k gt_ij = 2 D_kij).  The
    trace of At then changes by 3 lam and its gradient by 3 dlam.  In the first-order system
    the red terms turn that gradient into 6 alpha gt^ik dlam_k in the Ghat and b equations; in
    the second-order system they are absent, so only the remaining closed-form terms are left.
    The auxiliaries' right-hand sides are zero, and the other primaries equal the first-order
    ones exactly."""
    fo, so = orc.params(), orc.params(formulation=1)
    q, dq = _generic_point(seed)
    rng = np.random.default_rng(100 + seed)
    lam = 0.13
    dlam = rng.normal(size=3) * 0.2
    gt = np.array([[q[s_sym(i, j)] for j in range(3)] for i in range(3)])
    D = np.array([[[q[37 + 6 * k + s_sym(i, j)] for j in range(3)] for i in range(3)] for k in range(3)])
    q2, dq2 = q.copy(), dq.copy()
    for n_, (i, j) in enumerate(SYM):
        q2[11 + n_] += lam * gt[i, j]
        for k in range(3):
            dq2[k, 11 + n_] += dlam[k] * gt[i, j] + 2 * lam * D[k, i, j]
    r1, r2 = orc.rhs_point(so, q, dq), orc.rhs_point(so, q2, dq2)
    d = r2 - r1
    al, phi, A, P = q[6], q[10], q[25:28], q[55:58]
    ig = np.linalg.inv(gt)
    Gt = np.einsum("jk,il,jkl->i", ig, ig, D) + np.einsum("jk,il,kjl->i", ig, ig, D) - np.einsum(
        "jk,il,ljk->i", ig, ig, D)
    expG = 2 * al * lam * Gt - 6 * al * lam * ig @ P / phi - 2 * lam * ig @ A
    np.testing.assert_allclose(d[19:22], expG, atol=1e-12)
    np.testing.assert_allclose(d[22:25], expG, atol=1e-12)
    assert np.all(r1[25:58] == 0.0) and np.all(r2[25:58] == 0.0)
    # the primaries other than Ghat and b see no red term at all
    f1 = orc.rhs_point(fo, q, dq)
    keep = list(range(0, 19)) + [58]
    assert np.array_equal(r1[keep], f1[keep])


def _rhs_error(Qf, pr, center, h):
    Q, dt = ex.evaluate(Qf, box_points(center, h), with_dt=True)
    out = orc.rhs_box(pr, [h, h, h], Q)
    I = slice(3, 12)
    return np.abs(out[I, I, I] - dt[I, I, I]).reshape(-1, 59).max(0), out


def _assert_fourth_order(e1, e2, comps, floor):
    big = [c for c in comps if e1[c] > floor]
    assert big, "nothing to measure"
    assert max(e1[c] for c in comps) / max(e2[c] for c in comps) > 12.0
    for c in big:
        assert e1[c] / e2[c] > 12.0, (c, e1[c], e2[c])


def test_so_rhs_gauge_wave_exact_time_derivative():
    """Gauge wave along a generic direction, harmonic slicing, zero shift: the right-hand
    sides of the 24 primaries converge to the exact d_t Q at fourth order; A, B, D, P get 0."""
    Qf = ex.ccz4_from_adm(ex.adm_from_g4(ex.g4_gauge_wave(0.1, 2.0, (1, 2, 3))))
    pr = orc.params(kappa1=1.0, kappa2=0.0, kappa3=0.0, ko_eps=0.1, slicing=0, shift=0, formulation=1)
    e1, o1 = _rhs_error(Qf, pr, (0.13, 0.21, -0.17), 0.04)
    e2, _ = _rhs_error(Qf, pr, (0.13, 0.21, -0.17), 0.02)
    _assert_fourth_order(e1, e2, list(range(25)), 1e-9)
    assert np.all(o1[3:12, 3:12, 3:12, 25:58] == 0.0)


def test_so_rhs_static_schwarzschild_vanishes():
    """Static Schwarzschild, 1+log slicing and Gamma-driver: the primaries' right-hand sides
    tend to 0 at fourth order in the second-order formulation as well."""
    Qf = ex.ccz4_from_adm(ex.adm_from_g4(ex.g4_schwarzschild_isotropic(1.0)))
    pr = orc.params(formulation=1)
    e1, _ = _rhs_error(Qf, pr, (2.1, 1.3, -1.7), 0.04)
    e2, _ = _rhs_error(Qf, pr, (2.1, 1.3, -1.7), 0.02)
    _assert_fourth_order(e1, e2, list(range(25)), 1e-10)
    assert e2[:25].max() < 2e-9


@pytest.mark.slow
def test_so_gauge_wave_rk4_converges_to_exact_solution():
    """The gauge-wave benchmark in the second-order formulation (Algorithm 2 with RK4): the
    primaries after T converge to the exact wave at fourth order, and every auxiliary equals
    the FD4 reconstruction from the primaries after each step."""
    A, k = 0.1, 2.0
    Qf = ex.ccz4_from_adm(ex.adm_from_g4(ex.g4_gauge_wave(A, k, (1, 0, 0))))
    pr = orc.params(kappa1=1.0, kappa2=0.0, kappa3=0.0, ko_eps=0.1, slicing=0, shift=0, formulation=1)
    T = 8 * 0.1 / 27
    errs = []
    for npx in (3, 6):
        h = 1.0 / (9 * npx)
        m = orc.Mesh([npx, 1, 1], [-0.5, 0, 0], [1.0, 9 * h, 9 * h], bc=0)
        Q = m.zeros()
        m.init(Q, 0, [A, k])
        m.fill_halos(Q)
        m.reconstruct(Q)
        for _ in range(int(round(T / (0.1 * h)))):
            Q = m.rk4_step(pr, Q, 0.1 * h)
        R = Q.copy()
        m.fill_halos(R)
        m.reconstruct(R)
        I = (slice(None), slice(3, 12), slice(3, 12), slice(3, 12))
        assert np.array_equal(R[I], Q[I])
        err = 0.0
        for p in range(m.np):
            X = m.cell_centers(p)[3:12, 3:12, 3:12]
            Qx = ex.evaluate(Qf, X, t=T)
            err = max(err, np.abs(Q[p, 3:12, 3:12, 3:12, :25] - Qx[..., :25]).max())
        errs.append(err)
    assert errs[0] / errs[1] > 12.0, errs
    assert errs[1] < 1e-5

"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test checks the oracle against something other than itself: exact solutions of the
Einstein equations built independently from closed-form 4-metrics (tests/exact_ccz4.py),
values printed in the paper, closed forms of special cases, invariances, and the polynomial
exactness / Fourier symbols of the stencils.
"""
import math

import numpy as np
import pytest

import exact_ccz4 as ex
import oracle as orc
from seeded_inputs import box_points, smooth_state

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
GEOMETRIC = [0, 1, 2, 3, 4, 5, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21] + list(range(37, 58))


def s_sym(i, j):
    return SYM.index((min(i, j), max(i, j)))


# ------------------------------------------------------------------ stencils (App. D)

def test_fd4_exact_on_quartics_and_symbol():
    rng = np.random.default_rng(0)
    for deg in range(5):
        c = rng.normal(size=deg + 1)
        for dx in (0.1, 0.37):
            x0 = 0.3
            xs = x0 + dx * np.arange(-2, 3)
            v = np.polyval(c, xs)
            exact = np.polyval(np.polyder(c), x0) if deg else 0.0
            assert abs(orc.fd4(v, dx) - exact) < 1e-11 * (1 + abs(exact))
    # degree 5 is not exact: error = -dx^4/30 f^(5)
    dx = 0.1
    xs = dx * np.arange(-2, 3)
    assert abs(orc.fd4(xs ** 5, dx) - (-dx ** 4 / 30 * 120)) < 1e-10
    # Fourier symbol: i (8 sin t - sin 2t) / (6 dx)
    for th in (0.3, 1.1, 2.5):
        v = np.exp(1j * th * np.arange(-2, 3))
        re = orc.fd4(v.real, dx)
        im = orc.fd4(v.imag, dx)
        assert abs((re + 1j * im) - 1j * (8 * np.sin(th) - np.sin(2 * th)) / (6 * dx)) < 1e-12 / dx


def test_ko_annihilates_quintics_and_symbol():
    rng = np.random.default_rng(1)
    for deg in range(6):
        c = rng.normal(size=deg + 1)
        xs = 0.2 + 0.15 * np.arange(-3, 4)
        assert abs(orc.ko(np.polyval(c, xs), 0.15, 0.7)) < 1e-10
    # sixth difference of x^6 is 6! dx^6 -> KO = eps/(64 dx) * 720 dx^6
    dx, eps = 0.1, 0.3
    xs = dx * np.arange(-3, 4)
    assert abs(orc.ko(xs ** 6, dx, eps) - eps / (64 * dx) * 720 * dx ** 6) < 1e-14
    # symbol -eps (2 sin(t/2))^6 / (64 dx): dissipative
    for th in (0.4, 1.7, math.pi):
        v = np.cos(th * np.arange(-3, 4))
        assert abs(orc.ko(v, dx, eps) - (-eps * (2 * np.sin(th / 2)) ** 6 / (64 * dx))) < 1e-12


# ------------------------------------------------------------------ initial data

def test_gauge_wave_init_matches_paper_closed_forms():
    """alpha = sqrt(H), phi = H^(-1/6), K_xx = -(k pi A/2) cos / H^(1/2), K = K_xx / H, and the
    whole 59-vector equals the state built from the 4-metric ds^2 = -H dt^2 + H dx^2 + dy^2 + dz^2."""
    A, k = 0.1, 2.0
    Qf = ex.ccz4_from_adm(ex.adm_from_g4(ex.g4_gauge_wave(A, k, (1, 0, 0))))
    pts = np.random.default_rng(2).uniform(-0.5, 0.5, (16, 3))
    Qx = ex.evaluate(Qf, pts)
    for p, qx in zip(pts, Qx):
        q = orc.init_point(0, [A, k], p)
        Hh = 1 - A * math.sin(k * math.pi * p[0])
        Kxx = -k * math.pi * A / 2 * math.cos(k * math.pi * p[0]) / math.sqrt(Hh)
        assert abs(q[6] - math.sqrt(Hh)) < 1e-15
        assert abs(q[10] - Hh ** (-1 / 6)) < 1e-15
        assert abs(q[17] - Kxx / Hh) < 1e-14
        # At_xx = phi^2 (K_xx - K gamma_xx / 3)
        assert abs(q[11] - Hh ** (-1 / 3) * (Kxx - Kxx / Hh * Hh / 3)) < 1e-14
        assert np.abs(q - qx).max() < 1e-13


@pytest.mark.parametrize("lapse,kind", [("psi-2", 0), ("average", 1), ("static", 2)])
def test_puncture_init_matches_definitions(lapse, kind):
    Qf = ex.ccz4_from_adm(ex.adm_puncture(1.0, (0.1, -0.2, 0.05), lapse))
    pts = np.random.default_rng(3).uniform(-3, 3, (16, 3))
    Qx = ex.evaluate(Qf, pts)
    for p, qx in zip(pts, Qx):
        q = orc.init_point(1, [1.0, 0.1, -0.2, 0.05, kind], p)
        assert np.abs(q - qx).max() < 1e-12 * max(1, np.abs(qx).max())


def test_brill_lindquist_bowen_york_init_matches_definitions():
    holes = [(0.5, (3.0, 0.0, 0.0), (0.0, 0.095, 0.0)), (0.5, (-3.0, 0.0, 0.0), (0.0, -0.095, 0.0))]
    sp = [0.5, 3, 0, 0, 0, 0.095, 0, 0.5, -3, 0, 0, 0, -0.095, 0]
    Qf = ex.ccz4_from_adm(ex.adm_brill_lindquist_bowen_york(holes))
    pts = np.random.default_rng(4).uniform(-6, 6, (16, 3))
    Qx = ex.evaluate(Qf, pts)
    for p, qx in zip(pts, Qx):
        q = orc.init_point(2, sp, p)
        assert np.abs(q - qx).max() < 1e-12 * max(1, np.abs(qx).max())


# ------------------------------------------------------------------ RHS on exact solutions

def _rhs_error(Qf, pr, center, h):
    pts = box_points(center, h)
    Q, dt = ex.evaluate(Qf, pts, with_dt=True)
    out = orc.rhs_box(pr, [h, h, h], Q)
    I = slice(3, 12)
    return np.abs(out[I, I, I] - dt[I, I, I]).reshape(-1, 59).max(0), Q, dt, out


def _assert_fourth_order(e1, e2, comps, floor):
    """The discrete RHS of exact data converges to the exact d_t Q at fourth order (KO adds
    O(h^5)): halving h shrinks the worst error by about 16 or more."""
    big = [c for c in comps if e1[c] > floor]
    assert big, "nothing to measure"
    worst1 = max(e1[c] for c in comps)
    worst2 = max(e2[c] for c in comps)
    assert worst1 / worst2 > 12.0, (worst1, worst2)
    for c in big:
        assert e1[c] / e2[c] > 12.0, (c, e1[c], e2[c])


GW_PARAMS = dict(kappa1=1.0, kappa2=0.0, kappa3=0.0, e=1.0, c=1.0, tau=1.0, mu=0.2,
                 ko_eps=0.1, slicing=0, shift=0)


@pytest.mark.parametrize("n", [(1, 0, 0), (1, 2, 3)])
def test_rhs_gauge_wave_exact_time_derivative(n):
    """Gauge wave (harmonic slicing, zero shift) along x and along a generic direction:
    the 58 right-hand sides converge to the exact d_t Q at fourth order."""
    Qf = ex.ccz4_from_adm(ex.adm_from_g4(ex.g4_gauge_wave(0.1, 2.0, n)))
    pr = orc.params(**GW_PARAMS)
    e1 = _rhs_error(Qf, pr, (0.13, 0.21, -0.17), 0.04)[0]
    e2 = _rhs_error(Qf, pr, (0.13, 0.21, -0.17), 0.02)[0]
    _assert_fourth_order(e1, e2, list(range(58)), 1e-9)
    assert e2.max() < 2e-4


def test_rhs_static_schwarzschild_vanishes():
    """Static Schwarzschild in isotropic coordinates with 1+log slicing and the Gamma-driver:
    every exact time derivative is zero; the discrete RHS tends to 0 at fourth order."""
    Qf = ex.ccz4_from_adm(ex.adm_from_g4(ex.g4_schwarzschild_isotropic(1.0)))
    pr = orc.params()
    e1 = _rhs_error(Qf, pr, (2.1, 1.3, -1.7), 0.04)[0]
    e2 = _rhs_error(Qf, pr, (2.1, 1.3, -1.7), 0.02)[0]
    _assert_fourth_order(e1, e2, list(range(58)), 1e-10)
    assert e2.max() < 2e-9


def test_rhs_distorted_minkowski_geometric_sector_and_gauge_consistency():
    """Minkowski space in distorted coordinates: generic lapse, shift, metric and extrinsic
    curvature.  The geometric right-hand sides converge to the exact d_t Q; the gauge
    right-hand sides are consistent with the auxiliaries' definitions (A = d alpha,
    B = d beta): RHS(A_k) -> d_k RHS(alpha), RHS(B_k^i) -> d_k RHS(beta^i), and
    RHS(b) -> d_t Ghat - beta.d Ghat (b = 0)."""
    import torch
    from torch.func import jacfwd, vmap
    adm = ex.adm_from_g4(ex.g4_distorted_minkowski(0.05))
    Qf = ex.ccz4_from_adm(adm)
    pr = orc.params(slicing=1, shift=1, f=0.75, eta=2.0)
    center = (0.13, 0.21, -0.17)
    errs = []
    for h in (0.04, 0.02):
        e, Q, dt, out = _rhs_error(Qf, pr, center, h)
        pts = box_points(center, h)[3:12, 3:12, 3:12].reshape(-1, 3)

        def rhs_alpha_beta(X):
            q = Qf(X)
            al, beta, Kt, A, B = q[6], q[7:10], q[17], q[25:28], q[28:37].reshape(3, 3)
            g = 2.0 / al
            ra = beta @ A - al * al * g * Kt
            rb = beta @ B + pr.f * q[22:25]
            return torch.cat([ra.reshape(1), rb])

        X = torch.zeros((pts.shape[0], 4))
        X[:, 1:] = torch.from_numpy(pts)
        J = vmap(jacfwd(rhs_alpha_beta))(X).numpy()   # (n, 4, 4): [out, coord]
        grad_ra = J[:, 0, 1:]                          # d_k RHS(alpha)
        grad_rb = np.transpose(J[:, 1:, 1:], (0, 2, 1))  # [k, i] = d_k RHS(beta^i)
        o = out[3:12, 3:12, 3:12].reshape(-1, 59)
        Qi = Q[3:12, 3:12, 3:12].reshape(-1, 59)
        dti = dt[3:12, 3:12, 3:12].reshape(-1, 59)
        _, dQ = ex.evaluate(Qf, pts, with_dx=True)     # (n, 3, 59)
        beta = Qi[:, 7:10]
        adv_ghat = np.einsum("nk,nki->ni", beta, dQ[:, :, 19:22])
        eA = np.abs(o[:, 25:28] - grad_ra).max()
        eB = np.abs(o[:, 28:37] - grad_rb.reshape(-1, 9)).max()
        eb = np.abs(o[:, 22:25] - (dti[:, 19:22] - adv_ghat)).max()
        errs.append((e, eA, eB, eb))
    (e1, a1, B1, b1), (e2, a2, B2, b2) = errs
    _assert_fourth_order(e1, e2, GEOMETRIC, 1e-10)
    for x1, x2 in ((a1, a2), (B1, B2), (b1, b2)):
        assert x1 / x2 > 12.0, (x1, x2)
        assert x2 < 1e-6


# ------------------------------------------------------------------ closed forms at a point

def _homog_state(rng, alpha=1.3, Theta=0.2, K=-0.4, phi=1.0):
    q = np.zeros(59)
    q[[0, 3, 5]] = 1.0
    q[6] = alpha
    q[7:10] = rng.normal(size=3) * 0.3
    q[10] = phi
    At = rng.normal(size=(3, 3)) * 0.2
    At = 0.5 * (At + At.T)
    At -= np.trace(At) / 3 * np.eye(3)
    q[11:17] = [At[i, j] for (i, j) in SYM]
    q[17] = K
    q[18] = Theta
    q[19:22] = rng.normal(size=3) * 0.3
    q[22:25] = rng.normal(size=3) * 0.3
    q[25:28] = rng.normal(size=3) * 0.3
    q[28:37] = rng.normal(size=9) * 0.3
    return q, At


@pytest.mark.parametrize("slicing,shift", [(0, 0), (1, 1)])
def test_homogeneous_state_closed_form(slicing, shift):
    """Flat conformal metric, phi = 1, D = P = 0 and every derivative zero: the right-hand
    side reduces to the algebraic source terms, written out here for this special case."""
    rng = np.random.default_rng(5)
    pr = orc.params(kappa1=0.3, kappa2=0.4, kappa3=0.7, tau=2.0, e=1.5, c=0.8, mu=0.2, f=0.75,
                    eta=1.7, slicing=slicing, shift=shift)
    q, At = _homog_state(rng)
    if not shift:
        q[7:10] = 0
        q[22:25] = 0
        q[28:37] = 0
    al, Th, K, beta, Ghat, b, A = q[6], q[18], q[17], q[7:10], q[19:22], q[22:25], q[25:28]
    B = q[28:37].reshape(3, 3)  # B[k, i] = d_k beta^i
    trB = np.trace(B)
    g, gp = (2 / al, -2 / al ** 2) if slicing else (1.0, 0.0)
    s = 1.0 if shift else 0.0
    Z = 0.5 * Ghat
    out = orc.rhs_point(pr, q, np.zeros((3, 59)))
    exp = np.zeros(59)
    gtr = B.T + B - 2 / 3 * np.eye(3) * trB - 2 * al * At    # B_j^i + B_i^j = B[j,i] + B[i,j]
    exp[0:6] = [gtr[i, j] for (i, j) in SYM]
    exp[6] = beta @ A - al ** 2 * g * (K - 2 * pr.c * Th)
    exp[7:10] = s * (beta @ B + pr.f * b)
    exp[10] = (al * K - trB) / 3
    Atr = At.T @ B.T + (At.T @ B.T).T - 2 / 3 * At * trB + al * At * (K - 2 * Th * pr.c) - 2 * al * At @ At
    exp[11:17] = [Atr[i, j] for (i, j) in SYM]
    exp[17] = al * K * (K - 2 * Th * pr.c) - 3 * al * pr.kappa1 * (1 + pr.kappa2) * Th
    exp[18] = (0.5 * al * pr.e ** 2 * (2 / 3 * K ** 2 - np.sum(At * At)) - al * Th * K * pr.c
               - Z @ A - al * pr.kappa1 * (2 + pr.kappa2) * Th)
    rG = (-2 * Th * A - 4 / 3 * al * K * Z - 2 * At @ A - 2 * al * pr.kappa1 * Z
          + 2 * pr.kappa3 * (2 / 3 * Z * trB - Z @ B))
    exp[19:22] = rG
    exp[22:25] = s * (rG - pr.eta * b)
    exp[25:28] = B @ A - (2 * al * g + al ** 2 * gp) * (K - 2 * pr.c * Th) * A
    exp[28:37] = s * (B @ B).reshape(-1)
    for k in range(3):
        for n_, (i, j) in enumerate(SYM):
            exp[37 + 6 * k + n_] = -A[k] * At[i, j]
    exp[55:58] = K * A / 3
    np.testing.assert_allclose(out, exp, rtol=0, atol=1e-14)


def test_metric_determinant_relaxation():
    """gt = lambda delta (det = lambda^3), everything else trivial: d_t gt = -(det - 1) gt / tau."""
    pr = orc.params(tau=0.7)
    for lam in (0.9, 1.0, 1.2):
        q = np.zeros(59)
        q[[0, 3, 5]] = lam
        q[6] = 1.0
        q[10] = 1.0
        out = orc.rhs_point(pr, q, np.zeros((3, 59)))
        exp = -(lam ** 3 - 1) * lam / pr.tau
        np.testing.assert_allclose(out[[0, 3, 5]], exp, atol=1e-15)
        assert np.abs(np.delete(out, [0, 3, 5])).max() < 1e-15


def test_homogeneous_with_gradients_closed_form():
    """Flat conformal metric, phi = 1, D = P = 0, with constant gradients of Ghat, K, Theta and
    the advected fields: the Z4 terms R + 2 nabla Z = div Ghat and the gradient sources."""
    rng = np.random.default_rng(6)
    pr = orc.params(kappa1=0.3, kappa2=0.4, kappa3=0.7, e=1.5, c=0.8, slicing=1, shift=1)
    q, At = _homog_state(rng)
    dq = np.zeros((3, 59))
    dG = rng.normal(size=(3, 3)) * 0.3   # dG[k, i] = d_k Ghat^i
    dK = rng.normal(size=3) * 0.3
    dT = rng.normal(size=3) * 0.3
    dq[:, 19:22] = dG
    dq[:, 17] = dK
    dq[:, 18] = dT
    out = orc.rhs_point(pr, q, dq)
    ref = orc.rhs_point(pr, q, np.zeros((3, 59)))
    al, beta, phi = q[6], q[7:10], q[10]
    g = 2 / al
    div = np.trace(dG)
    d = out - ref
    np.testing.assert_allclose(d[17], beta @ dK + al * div, atol=1e-14)
    np.testing.assert_allclose(d[18], beta @ dT + 0.5 * al * pr.e ** 2 * div, atol=1e-14)
    X = al * 0.5 * (dG + dG.T)
    Xtf = X - np.trace(X) / 3 * np.eye(3)
    np.testing.assert_allclose(d[11:17], [Xtf[i, j] for (i, j) in SYM], atol=1e-14)
    np.testing.assert_allclose(d[19:22], beta @ dG + 2 * al * dT - 4 / 3 * al * dK, atol=1e-14)
    np.testing.assert_allclose(d[22:25], 2 * al * dT - 4 / 3 * al * dK, atol=1e-14)  # advection cancels
    np.testing.assert_allclose(d[25:28], -al ** 2 * g * (dK - 2 * pr.c * dT), atol=1e-14)
    np.testing.assert_allclose(d[55:58], phi * al * dK / 3, atol=1e-14)
    untouched = [i for i in range(59) if i not in (list(range(11, 28)) + [55, 56, 57])]
    assert np.abs(d[untouched]).max() < 1e-14


def _generic_point(seed):
    rng = np.random.default_rng(seed)
    q = smooth_state(rng.uniform(-1, 1, (1, 3)), seed)[0]
    dq = rng.normal(size=(3, 59)) * 0.2
    return q, dq


def _gt(q):
    return np.array([[q[s_sym(i, j)] for j in range(3)] for i in range(3)])


def _D(q):
    return np.array([[[q[37 + 6 * k + s_sym(i, j)] for j in range(3)] for i in range(3)] for k in range(3)])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_trace_constraint_terms(seed):
    """The constraint-addition (red) terms of App. B collapse via d_k gt^nm = -2 D_k^nm to
    multiples of d_k (tr At).  Shifting At -> At + lam gt (with d At shifted consistently,
    d_k gt_ij = 2 D_kij) changes the right-hand sides by closed forms, for any state."""
    pr = orc.params()
    q, dq = _generic_point(seed)
    rng = np.random.default_rng(100 + seed)
    lam = 0.13
    dlam = rng.normal(size=3) * 0.2
    gt, D = _gt(q), _D(q)
    q2, dq2 = q.copy(), dq.copy()
    for n_, (i, j) in enumerate(SYM):
        q2[11 + n_] += lam * gt[i, j]
        for k in range(3):
            dq2[k, 11 + n_] += dlam[k] * gt[i, j] + 2 * lam * D[k, i, j]
    d = orc.rhs_point(pr, q2, dq2) - orc.rhs_point(pr, q, dq)
    al, phi, A, P = q[6], q[10], q[25:28], q[55:58]
    ig = np.linalg.inv(gt)
    g = 2 / al
    # Gt^i = gt^jk gt^il (D_jkl + D_kjl - D_ljk)
    Gt = np.einsum("jk,il,jkl->i", ig, ig, D) + np.einsum("jk,il,kjl->i", ig, ig, D) - np.einsum(
        "jk,il,ljk->i", ig, ig, D)
    At = np.array([[q[11 + s_sym(i, j)] for j in range(3)] for i in range(3)])
    trAt = np.sum(ig * At)
    np.testing.assert_allclose(d[25:28], -3 * al * g * dlam, atol=1e-13)
    np.testing.assert_allclose(d[55:58], al * phi * dlam, atol=1e-13)
    for k in range(3):
        for n_, (i, j) in enumerate(SYM):
            assert abs(d[37 + 6 * k + n_] - (-2 * al * lam * D[k, i, j])) < 1e-13
    expG = 6 * al * ig @ dlam + 2 * al * lam * Gt - 6 * al * lam * ig @ P / phi - 2 * lam * ig @ A
    np.testing.assert_allclose(d[19:22], expG, atol=1e-12)
    np.testing.assert_allclose(d[22:25], expG, atol=1e-12)
    np.testing.assert_allclose(d[0:6], 0, atol=1e-13)
    np.testing.assert_allclose(d[17], 0, atol=1e-13)
    np.testing.assert_allclose(d[18], -0.5 * al * pr.e ** 2 * (2 * lam * trAt + 3 * lam ** 2), atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_curl_terms_and_advection(seed):
    """Antisymmetric (curl) parts of the derivatives of the auxiliaries.  Symmetrised
    derivatives (Ricci, nabla nabla alpha, d_(k B_l)) do not see them; they enter only the
    mu terms of the B equation and the advection terms beta^l d_l of A, B, D, P."""
    pr = orc.params(mu=0.37)
    q, dq = _generic_point(seed)
    rng = np.random.default_rng(200 + seed)
    al, phi, beta = q[6], q[10], q[7:10]
    ig = np.linalg.inv(_gt(q))
    w = rng.normal(size=(3, 3))
    w = w - w.T                                   # curl of P: d_k P_j += w[k, j]
    dq2 = dq.copy()
    dq2[:, 55:58] += w
    d = orc.rhs_point(pr, q, dq2) - orc.rhs_point(pr, q, dq)
    expB = -al ** 2 * pr.mu / phi * np.einsum("ij,kj->ki", ig, w - w.T)
    np.testing.assert_allclose(d[28:37], expB.reshape(-1), atol=1e-12)
    np.testing.assert_allclose(d[55:58], beta @ w, atol=1e-13)
    assert np.abs(np.delete(d, list(range(28, 37)) + [55, 56, 57])).max() < 1e-13
    # curl of D: d_k D_ljn += W[k, l, j, n], antisymmetric in (k, l), symmetric in (j, n)
    W = rng.normal(size=(3, 3, 3, 3))
    W = W - W.transpose(1, 0, 2, 3)
    W = W + W.transpose(0, 1, 3, 2)
    dq3 = dq.copy()
    for k in range(3):
        for l in range(3):
            for n_, (j, n) in enumerate(SYM):
                dq3[k, 37 + 6 * l + n_] += W[k, l, j, n]
    d = orc.rhs_point(pr, q, dq3) - orc.rhs_point(pr, q, dq)
    expB = al ** 2 * pr.mu * np.einsum("ij,nl,kljn->ki", ig, ig, W - W.transpose(1, 0, 2, 3))
    np.testing.assert_allclose(d[28:37], expB.reshape(-1), atol=1e-12)
    expD = np.einsum("l,lkjn->kjn", beta, W)
    for k in range(3):
        for n_, (j, n) in enumerate(SYM):
            assert abs(d[37 + 6 * k + n_] - expD[k, j, n]) < 1e-13
    assert np.abs(np.delete(d, list(range(28, 37)) + list(range(37, 55)))).max() < 1e-13
    # curl of A and of B: only their own advection terms
    wa = rng.normal(size=(3, 3))
    wa = wa - wa.T
    dq4 = dq.copy()
    dq4[:, 25:28] += wa
    d = orc.rhs_point(pr, q, dq4) - orc.rhs_point(pr, q, dq)
    np.testing.assert_allclose(d[25:28], beta @ wa, atol=1e-13)
    assert np.abs(np.delete(d, [25, 26, 27])).max() < 1e-13
    wb = rng.normal(size=(3, 3, 3))
    wb = wb - wb.transpose(1, 0, 2)             # d_k B_l^i += wb[k, l, i]
    dq5 = dq.copy()
    dq5[:, 28:37] += wb.reshape(3, 9)
    d = orc.rhs_point(pr, q, dq5) - orc.rhs_point(pr, q, dq)
    np.testing.assert_allclose(d[28:37], np.einsum("l,lki->ki", beta, wb).reshape(-1), atol=1e-13)
    assert np.abs(np.delete(d, list(range(28, 37)))).max() < 1e-13


# ------------------------------------------------------------------ invariances

def _perm_tensor_slots(perm, sign):
    """Map slot -> (new slot, factor) under x_a -> sign_a x_perm(a)."""
    P = np.zeros((3, 3))
    for a in range(3):
        P[perm[a], a] = sign[a]
    return P


def transform_state(q, M):
    """Apply the linear coordinate change x' = M x (orthogonal, axis permutation/reflection)
    to every tensor slot of the 59-vector (vectors, one-forms and derivatives alike)."""
    out = q.copy()
    g = np.array([[q[s_sym(i, j)] for j in range(3)] for i in range(3)])
    At = np.array([[q[11 + s_sym(i, j)] for j in range(3)] for i in range(3)])
    gp, Ap = M @ g @ M.T, M @ At @ M.T
    for n_, (i, j) in enumerate(SYM):
        out[n_], out[11 + n_] = gp[i, j], Ap[i, j]
    for base in (7, 19, 22, 25, 55):
        out[base:base + 3] = M @ q[base:base + 3]
    out[28:37] = (M @ q[28:37].reshape(3, 3) @ M.T).reshape(-1)
    D = _D(q)
    Dp = np.einsum("ka,ib,jc,abc->kij", M, M, M, D)
    for k in range(3):
        for n_, (i, j) in enumerate(SYM):
            out[37 + 6 * k + n_] = Dp[k, i, j]
    return out


@pytest.mark.parametrize("perm,sign", [((1, 2, 0), (1, 1, 1)), ((0, 1, 2), (-1, 1, 1)),
                                       ((2, 0, 1), (1, -1, -1))])
def test_rhs_covariant_under_axis_permutation_and_reflection(perm, sign):
    """RHS(T Q) = T RHS(Q) for the orthogonal maps that carry the grid onto itself; the
    box is transformed as an array, so the stencils see exactly the transformed data."""
    M = _perm_tensor_slots(perm, sign)
    pr = orc.params()
    h = 0.05
    Q = smooth_state(box_points((0.1, -0.2, 0.3), h), 7)
    out = orc.rhs_box(pr, [h, h, h], Q)
    # array transform: new[z',y',x'] = old at x = M^T x'
    Xp = np.arange(15) - 7
    Qt = np.zeros_like(Q)
    outt_exp = np.zeros_like(Q)
    for iz in range(15):
        for iy in range(15):
            for ix in range(15):
                xp = np.array([Xp[ix], Xp[iy], Xp[iz]])
                x = M.T @ xp
                src = tuple(int(v) + 7 for v in x[::-1])
                Qt[iz, iy, ix] = transform_state(Q[src], M)
                outt_exp[iz, iy, ix] = transform_state(out[src], M)
    outt = orc.rhs_box(pr, [h, h, h], Qt)
    I = slice(3, 12)
    scale = np.abs(out[I, I, I]).reshape(-1, 59).max(0) + 1e-30
    err = np.abs(outt[I, I, I] - outt_exp[I, I, I]).reshape(-1, 59).max(0) / scale
    assert err.max() < 1e-12, (err.argmax(), err.max())

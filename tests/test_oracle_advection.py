"""Pins of the oracle's lopsided advection (App. D: the two one-sided-biased fourth-order
five-point stencils for the advection terms beta^k d_k Q): exactness on quartics and the
closed-form error on quintics, mirror symmetry of the pair, which grid points each pairing
reads (the upwind reading and the pairing as printed), and fourth-order convergence of the
right-hand side on an exact spacetime with a generic shift."""
import numpy as np
import pytest

import exact_ccz4 as ex
import oracle as orc
from seeded_inputs import box_points, smooth_state

GEOMETRIC = [0, 1, 2, 3, 4, 5, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20, 21] + list(range(37, 58))


@pytest.mark.parametrize("right", [0, 1])
def test_lopsided_exact_on_quartics_and_quintic_error(right):
    rng = np.random.default_rng(3 + right)
    for deg in range(5):
        c = rng.normal(size=deg + 1)
        for dx in (0.1, 0.37):
            x0 = -0.2
            v = np.polyval(c, x0 + dx * np.arange(-3, 4))
            exact = np.polyval(np.polyder(c), x0) if deg else 0.0
            assert abs(orc.fd4_lop(v, dx, right) - exact) < 1e-11 * (1 + abs(exact))
    # x^5 at 0: both stencils give 72 dx^5 / (12 dx) = 6 dx^4 = (dx^4 / 20) f^(5)
    dx = 0.1
    assert abs(orc.fd4_lop((dx * np.arange(-3, 4)) ** 5, dx, right) - 6 * dx ** 4) < 1e-13


def test_lopsided_pair_is_mirror_symmetric_and_reads_five_points():
    rng = np.random.default_rng(5)
    v = rng.normal(size=7)
    dx = 0.23
    assert abs(orc.fd4_lop(v, dx, 0) + orc.fd4_lop(v[::-1], dx, 1)) < 1e-14
    # the right-biased stencil never reads Q---, the left-biased one never Q+++
    for right, unused in ((1, 0), (0, 6)):
        w = v.copy()
        w[unused] += 1.0
        assert orc.fd4_lop(w, dx, right) == orc.fd4_lop(v, dx, right)


def _box_with_shift(beta):
    """A smooth random state on one box with a constant shift (so the pairing is fixed per axis)."""
    P = box_points((0.1, -0.2, 0.3), 0.05)
    Q = smooth_state(P, 11)
    Q[..., 7:10] = beta
    return Q


@pytest.mark.parametrize("mode", [1, 2])
def test_pairing_decides_which_far_point_the_advection_reads(mode):
    """Perturb K at the points 3 cells away from the box centre along each axis.  The central FD4
    of K reaches 2 cells only, so K's own right-hand side changes by the KO weight eps/(64 dx)
    plus, if the advection stencil along that axis reaches the point, beta^a times its App. D
    coefficient (1/(12 dx) at +3 for the right-biased stencil, -1/(12 dx) at -3 for the
    left-biased one).  Mode 1 takes the stencil biased towards +x_a where beta^a > 0, mode 2
    (as printed) towards -x_a there.  No other slot's right-hand side moves."""
    beta = np.array([0.3, -0.2, 0.45])
    Q = _box_with_shift(beta)
    dx = 0.05
    pr = orc.params(ko_eps=0.1, advection=mode)
    base = orc.rhs_box(pr, [dx] * 3, Q)[7, 7, 7]
    delta = 1e-3
    for a in range(3):
        for side in (-1, 1):
            Qp = Q.copy()
            idx = [7, 7, 7]
            idx[2 - a] += 3 * side  # [z, y, x] storage
            Qp[tuple(idx) + (17,)] += delta
            out = orc.rhs_box(pr, [dx] * 3, Qp)[7, 7, 7]
            right = (beta[a] > 0) if mode == 1 else not (beta[a] > 0)
            reach = (side > 0 and right) or (side < 0 and not right)
            expect = pr.ko_eps / (64 * dx) * delta
            if reach:
                expect += beta[a] * (1.0 if side > 0 else -1.0) * delta / (12 * dx)
            assert abs((out[17] - base[17]) - expect) < 1e-9 * abs(expect), (a, side, out[17] - base[17], expect)
            others = [v for v in range(59) if v != 17]
            assert np.array_equal(out[others], base[others])


@pytest.mark.parametrize("mode", [1, 2])
def test_lopsided_rhs_converges_on_distorted_minkowski(mode):
    """Minkowski space in distorted coordinates (generic lapse and shift): with either pairing the
    geometric right-hand sides still converge to the exact d_t Q at fourth order, and differ
    from the central-advection ones by a fourth-order amount."""
    adm = ex.adm_from_g4(ex.g4_distorted_minkowski(0.05))
    Qf = ex.ccz4_from_adm(adm)
    center = (0.13, 0.21, -0.17)
    pr = orc.params(slicing=1, shift=1, f=0.75, eta=2.0, advection=mode)
    pc = orc.params(slicing=1, shift=1, f=0.75, eta=2.0)
    errs, diffs = [], []
    I = slice(3, 12)
    for h in (0.04, 0.02):
        Q, dt = ex.evaluate(Qf, box_points(center, h), with_dt=True)
        out = orc.rhs_box(pr, [h] * 3, Q)[I, I, I].reshape(-1, 59)
        cen = orc.rhs_box(pc, [h] * 3, Q)[I, I, I].reshape(-1, 59)
        errs.append(np.abs(out - dt[I, I, I].reshape(-1, 59)).max(0))
        diffs.append(np.abs(out - cen).max(0))
    e1, e2 = errs
    big = [c for c in GEOMETRIC if e1[c] > 1e-10]
    assert big
    for c in big:
        assert e1[c] / e2[c] > 12.0, (c, e1[c], e2[c])
    d1, d2 = diffs
    adv = [c for c in range(11, 58) if d1[c] > 1e-10]
    assert adv  # the lopsided stencils do change the advected slots
    assert max(d1[adv]) / max(d2[adv]) > 12.0

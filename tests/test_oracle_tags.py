"""Pins of the oracle's plain refinement criterion (no GPU).

The paper's feature-based refinement (Sec. 3.6) refines a patch where the largest difference
between two adjacent volumes of the patch is large.  The readings here: the differences are
taken of chi = phi^2 and of alpha over face-adjacent interior cells, a constraint term
dx^2 max|H| joins them, e is the largest of the three; e >= theta_r refines (ties refine) below
max_level; a leaf of level >= 1 coarsens only when e < theta_c on it and on all 27 leaves of its
family; otherwise KEEP.

Each value checked below is a closed form of the state, not a re-evaluation of the criterion:
linear fields give the adjacent differences exactly, a homogeneous state gives H exactly
(every derivative vanishes, so R = 0 and H = 2/3 K^2 - At_ij At^ij), and hand-made
sibling families give the tags."""
import math

import numpy as np

import oracle as orc

SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
I = slice(3, 12)


def _flat_state(m, phi=1.0, alpha=1.0):
    """gt = delta, the given phi and alpha everywhere (halos too), every other slot 0."""
    Q = m.zeros()
    for s in (0, 3, 5):
        Q[..., s] = 1.0
    Q[..., 10] = phi
    Q[..., 6] = alpha
    return Q


def _homogeneous(Q, p, K, At, phi=0.8, alpha=0.9):
    """Leaf p's whole box (halos included) set to a homogeneous state: gt = delta, phi, alpha,
    K and the trace-free At constant; every derivative of it vanishes exactly."""
    Q[p] = 0.0
    for s in (0, 3, 5):
        Q[p, ..., s] = 1.0
    Q[p, ..., 10] = phi
    Q[p, ..., 6] = alpha
    Q[p, ..., 17] = K
    for s in range(6):
        Q[p, ..., 11 + s] = At[s]


def _hamiltonian_homogeneous(K, At):
    """H = R + 2/3 K^2 - At_ij At^ij with R = 0 and At raised by gt = delta."""
    AA = sum((1.0 if i == j else 2.0) * At[s] ** 2 for s, (i, j) in enumerate(SYM))
    return 2.0 / 3.0 * K * K - AA


def test_indicator_adjacent_differences_of_linear_chi_alpha():
    """phi and alpha linear in x, y, z: the adjacent differences along axis a are exact, and the
    indicator is max_a s_a dx (phi(c) + phi(c + e_a)) for chi = phi^2 (largest at the interior's
    far corner) and max_a |u_a| dx for alpha; the constraint term is 0 (R = 0, K = At = 0)."""
    m = orc.Mesh([2, 1, 1], [0.0, 0.0, 0.0], [2.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0], bc=1)
    Q = _flat_state(m)
    s = np.array([0.7, -0.4, 1.3])     # slopes of phi
    u = np.array([-0.25, 0.55, 0.35])  # slopes of alpha
    for p in range(m.np):
        X = m.cell_centers(p)
        Q[p, ..., 10] = 1.5 + X @ s
        Q[p, ..., 6] = 0.9 + X @ u
    ind = m.tag_indicator(Q)
    for p in range(m.np):
        org, dx = m.geom[p, :3], m.geom[p, 3]
        centres = org[:, None] + (np.arange(9) + 0.5)[None, :] * dx  # [axis, i]
        gc = 0.0
        for a in range(3):
            # phi(c) + phi(c + e_a) is largest where every other axis sits at its end that
            # raises phi, and along a at the pair nearest that end
            hi = np.array([centres[b, -1] if s[b] > 0 else centres[b, 0] for b in range(3)])
            lo = hi.copy()
            lo[a] -= math.copysign(dx, s[a])
            gc = max(gc, abs(s[a]) * dx * ((1.5 + hi @ s) + (1.5 + lo @ s)))
        ga = np.max(np.abs(u)) * dx
        np.testing.assert_allclose(ind[p, 0], gc, rtol=1e-12)
        np.testing.assert_allclose(ind[p, 1], ga, rtol=1e-12)
        assert ind[p, 2] == 0.0
        # chi = phi^2, not phi: the difference of phi alone would be max_a |s_a| dx
        assert abs(ind[p, 0] - np.max(np.abs(s)) * dx) > 0.5 * np.max(np.abs(s)) * dx


def test_indicator_only_face_adjacent_interior_pairs():
    """A jump of alpha between the interior and a halo layer does not count (the pairs are
    interior ones), and a checkerboard in the x-y plane gives the face-adjacent difference, not a
    diagonal one (diagonal neighbours of a checkerboard are equal)."""
    m = orc.Mesh([1, 1, 1], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0], bc=1)
    Q = _flat_state(m, alpha=1.0)
    Q[0, :3, :, :, 6] = 50.0  # halo layers below the interior
    Q[0, :, :, 12:, 6] = -50.0
    ind = m.tag_indicator(Q)
    assert ind[0, 1] == 0.0
    z, y, x = np.meshgrid(np.arange(15), np.arange(15), np.arange(15), indexing="ij")
    Q[0, ..., 6] = 1.0 + 0.125 * ((x + y) % 2)
    ind = m.tag_indicator(Q)
    assert ind[0, 1] == 0.125


def test_indicator_constraint_term_is_dx_squared_max_abs_H():
    """Homogeneous leaves: H = 2/3 K^2 - At_ij At^ij exactly, so the third indicator is
    dx^2 |H| with the leaf's own spacing (dx = 1/27 on level 0, 1/81 on level 1), and the two
    difference terms vanish."""
    m = orc.Mesh([3, 1, 1], [0.0, 0.0, 0.0], [1.0, 1.0 / 3.0, 1.0 / 3.0], bc=1, refined=[(0, 1, 0, 0)])
    Q = m.zeros()
    rng = np.random.default_rng(3)
    expect = []
    for p in range(m.np):
        K = rng.uniform(-2.0, 2.0)
        At = rng.uniform(-0.6, 0.6, 6)
        At[5] = -(At[0] + At[3])  # trace free with gt = delta
        _homogeneous(Q, p, K, At)
        expect.append(_hamiltonian_homogeneous(K, At))
    ind = m.tag_indicator(Q)
    assert any(h < 0 for h in expect) and any(h > 0 for h in expect)
    for p in range(m.np):
        dx = m.geom[p, 3]
        assert ind[p, 0] == 0.0 and ind[p, 1] == 0.0
        np.testing.assert_allclose(ind[p, 2], dx * dx * abs(expect[p]), rtol=1e-13)
    assert {round(1.0 / m.geom[p, 3]) for p in range(m.np)} == {27, 81}


def _family_mesh():
    """3^3 level-0 cubes on [0, 3]^3 with the centre cube refined: 26 level-0 leaves and one
    family of 27 level-1 leaves."""
    return orc.Mesh([3, 3, 3], [0.0, 0.0, 0.0], [3.0, 3.0, 3.0], bc=1, refined=[(0, 1, 1, 1)])


def _state_with_H(m, hvals):
    """Homogeneous leaves whose H is hvals[p] (via K alone: H = 2/3 K^2); the indicator of leaf
    p is then dx_p^2 hvals[p]."""
    Q = m.zeros()
    for p in range(m.np):
        _homogeneous(Q, p, math.sqrt(1.5 * hvals[p]), np.zeros(6))
    return Q


def test_tag_threshold_tie_refines():
    """e equal to theta_r refines; the next double above e as theta_r keeps."""
    m = _family_mesh()
    h = np.full(m.np, 1.0)
    Q = _state_with_H(m, h)
    e = m.tag_indicator(Q).max(axis=1)
    lev = m.ids[:, 0]
    p1 = int(np.flatnonzero(lev == 1)[0])
    theta = e[p1]
    tags = m.tag_refine(Q, theta, -1.0, 2)
    assert tags[p1] == 1
    tags = m.tag_refine(Q, np.nextafter(theta, np.inf), -1.0, 2)
    assert tags[p1] == 0
    # a value equal to theta_c does not coarsen (e < theta_c is strict)
    fam = np.flatnonzero(lev == 1)
    assert np.all(m.tag_refine(Q, 1e9, np.nextafter(theta, np.inf), 2)[fam] == -1)
    assert np.all(m.tag_refine(Q, 1e9, theta, 2)[fam] == 0)


def test_tag_max_level_cap():
    """A leaf at max_level is not refined however large e is; below it, it is."""
    m = _family_mesh()
    Q = _state_with_H(m, np.full(m.np, 4.0))
    lev = m.ids[:, 0]
    tags = m.tag_refine(Q, 1e-6, -1.0, 1)
    assert np.all(tags[lev == 0] == 1) and np.all(tags[lev == 1] == 0)
    tags = m.tag_refine(Q, 1e-6, -1.0, 2)
    assert np.all(tags == 1)
    tags = m.tag_refine(Q, 1e-6, -1.0, 0)
    assert np.all(tags == 0)


def test_tag_sibling_families():
    """Level-1 leaves coarsen only as a whole family below theta_c; one sibling at or above
    theta_c (KEEP) or tagged REFINE blocks the family; level-0 leaves never coarsen."""
    m = _family_mesh()
    lev = m.ids[:, 0]
    fam = np.flatnonzero(lev == 1)
    # indicator = dx^2 H with the leaf's cell spacing dx
    dx2 = m.geom[:, 3] ** 2
    h = 0.01 / dx2  # every indicator 0.01
    Q = _state_with_H(m, h)
    e = m.tag_indicator(Q).max(axis=1)
    np.testing.assert_allclose(e, 0.01, rtol=1e-13)
    tags = m.tag_refine(Q, 1.0, 0.1, 3)
    assert np.all(tags[fam] == -1) and np.all(tags[lev == 0] == 0)
    # one sibling between the thresholds: KEEP for the whole family
    h2 = h.copy()
    h2[fam[13]] = 0.5 / dx2[fam[13]]
    tags = m.tag_refine(_state_with_H(m, h2), 1.0, 0.1, 3)
    assert np.all(tags[fam] == 0)
    # one sibling above theta_r: it refines, its siblings keep
    h3 = h.copy()
    h3[fam[5]] = 2.0 / dx2[fam[5]]
    tags = m.tag_refine(_state_with_H(m, h3), 1.0, 0.1, 3)
    assert tags[fam[5]] == 1
    assert np.all(np.delete(tags[fam], 5) == 0)


def test_tag_family_with_a_refined_sibling_keeps():
    """When one cube of a family is refined further, its 26 leaf siblings cannot coarsen (a
    sibling is not a leaf), while the 27 finer leaves below it can."""
    m = orc.Mesh([3, 3, 3], [0.0, 0.0, 0.0], [3.0, 3.0, 3.0], bc=1, refined=[(0, 1, 1, 1), (1, 4, 4, 4)])
    lev = m.ids[:, 0]
    assert (lev == 1).sum() == 26 and (lev == 2).sum() == 27
    dx2 = m.geom[:, 3] ** 2
    Q = _state_with_H(m, 0.01 / dx2)
    tags = m.tag_refine(Q, 1.0, 0.1, 3)
    assert np.all(tags[lev == 1] == 0)
    assert np.all(tags[lev == 2] == -1)
    assert np.all(tags[lev == 0] == 0)


def test_tag_level_zero_never_coarsens():
    """A uniform level-0 mesh whose 27 cubes are all below theta_c keeps every leaf: level 0 has
    no parent to coarsen into."""
    m = orc.Mesh([3, 3, 3], [0.0, 0.0, 0.0], [3.0, 3.0, 3.0], bc=1)
    Q = _state_with_H(m, np.full(m.np, 1e-3))
    assert np.all(m.tag_refine(Q, 1.0, 0.5, 3) == 0)

"""Pins of the oracle's tracers (Sec. 3.8: trilinear projection from the 2^3 nearest cell centres,
explicit Euler motion) and puncture trackers (velocity -beta): exactness on multilinear fields,
the closed-form error on a quadratic, cell-centre values, the leaf lookup on an AMR mesh checked
geometrically, and Euler steps in constant and linear shift fields."""
import numpy as np
import pytest

import oracle as orc
from seeded_inputs import box_centers


def amr_mesh():
    return orc.Mesh((2, 2, 1), (-1.0, -1.0, -0.5), (2.0, 2.0, 1.0), 1, [(0, 0, 1, 0)])


def fill_global(m, f, slot):
    """Every box cell (halos included) of every leaf gets f at its centre."""
    Q = m.zeros()
    for p in range(m.np):
        P = box_centers(m.geom[p, :3], m.geom[p, 3:])
        Q[p, ..., slot] = f(P[..., 0], P[..., 1], P[..., 2])
    return Q


def interior_points(m, n, rng):
    lo = np.array([-1.0, -1.0, -0.5])
    return lo + rng.random((n, 3)) * np.array([2.0, 2.0, 1.0]) * 0.999


def test_find_leaf_matches_geometry():
    m = amr_mesh()
    rng = np.random.default_rng(0)
    for x in interior_points(m, 300, rng):
        p = m.find_leaf(x)
        assert p >= 0
        o, dx = m.geom[p, :3], m.geom[p, 3:]
        assert np.all(x >= o) and np.all(x < o + 9 * dx)
        others = [q for q in range(m.np) if q != p and np.all(x >= m.geom[q, :3]) and
                  np.all(x < m.geom[q, :3] + 9 * m.geom[q, 3:])]
        assert not others
    assert m.find_leaf(np.array([5.0, 0.0, 0.0])) == -1


def test_find_leaf_leaves_no_gap_at_faces():
    """Points on leaf faces and corners, and within rounding of them, lie in exactly one leaf:
    the lookup compares integer cube indices, so the leaves tile the domain without the gaps that
    a test against each leaf's own floating-point box can leave (a puncture tracker sitting at
    z = -3e-26 next to the face z = 0 of a leaf of edge 0.5 fell into such a gap)."""
    from paper_2406_11626_amd import scenarios
    w = scenarios.binary_tracking([2.0])
    m = orc.Mesh(w.n0, w.origin, w.extent, w.bc, w.refined)
    x = np.array([3.0, 5.711970443685167e-10, -3.4465858856376157e-26])
    p = m.find_leaf(x)
    # x - origin rounds the offset away: the point belongs to the leaf above the face, and to one
    assert p >= 0 and m.geom[p, 2] == 0.0
    m = amr_mesh()
    rng = np.random.default_rng(3)
    corners = np.unique(np.concatenate([m.geom[:, :3], m.geom[:, :3] + 9 * m.geom[:, 3:]]), axis=0)
    lo, hi = np.array([-1.0, -1.0, -0.5]), np.array([1.0, 1.0, 0.5])
    for c in corners:
        for _ in range(6):
            x = c + rng.choice([-1e-300, 0.0, 1e-300, -1e-17, 1e-17], size=3)
            p = m.find_leaf(x)
            if np.all(x > lo + 1e-12) and np.all(x < hi - 1e-12):
                assert p >= 0, x  # inner faces and corners: always in a leaf
            elif np.any(x < lo - 1e-12) or np.any(x > hi + 1e-12):
                assert p < 0, x
            if p >= 0:
                o, e = m.geom[p, :3], 9 * m.geom[p, 3:]
                assert np.all(x >= o - 1e-12) and np.all(x <= o + e + 1e-12)


def test_trilinear_exact_on_multilinear_fields():
    m = amr_mesh()
    rng = np.random.default_rng(1)
    c = rng.normal(size=8)

    def f(x, y, z):
        return c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * x * z + c[6] * y * z + c[7] * x * y * z

    Q = fill_global(m, f, 17)
    pts = interior_points(m, 400, rng)
    out = m.tracer_sample(Q, pts, [17])
    np.testing.assert_allclose(out[:, 0], f(pts[:, 0], pts[:, 1], pts[:, 2]), rtol=0, atol=1e-13)


def test_trilinear_near_leaf_edges_reads_no_edge_or_corner_halo_cell():
    """A fill writes face halos only.  Near an edge (two faces) or a corner (three faces) of a leaf
    some of the eight cells lie in an edge or corner region of the leaf's halo; they must come
    from the interiors of the same-level leaves that hold them.  With interiors set to a
    multilinear field, every halo cell NaN before the fill, the samples at points within half a
    cell of inner edges and corners are exact (a single NaN read would show)."""
    m = orc.Mesh((3, 3, 3), (0.0, 0.0, 0.0), (3.0, 3.0, 3.0), 0)
    rng = np.random.default_rng(7)
    c = rng.normal(size=8)

    def f(x, y, z):
        return c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * x * z + c[6] * y * z + c[7] * x * y * z

    Q = fill_global(m, f, 9)
    inner = np.zeros((15, 15, 15), bool)
    inner[3:12, 3:12, 3:12] = True
    Q[:, ~inner, :] = np.nan
    m.fill_halos(Q)
    assert np.isnan(Q[:, 1, 1, 5, 9]).all()  # an edge-region cell of every leaf stays unwritten
    h = 0.5 / 9  # half a cell
    pts = []
    for _ in range(60):
        e = rng.choice([1.0, 2.0], size=3) + rng.uniform(-h, h, size=3) * 0.999
        free = rng.integers(0, 3)
        e2 = e.copy()
        e2[free] = rng.uniform(0.2, 2.8)  # near an edge: two coordinates at inner faces
        pts += [e, e2]
    pts = np.array(pts)
    out = m.tracer_sample(Q, pts, [9])
    np.testing.assert_allclose(out[:, 0], f(pts[:, 0], pts[:, 1], pts[:, 2]), rtol=0, atol=1e-12)


def test_trilinear_error_closed_form_on_a_quadratic():
    """For f = x^2 the trilinear interpolant between centres x_i and x_i + h errs by exactly
    h^2 t (1 - t) at x = x_i + t h."""
    m = amr_mesh()
    Q = fill_global(m, lambda x, y, z: x * x, 6)
    rng = np.random.default_rng(2)
    pts = interior_points(m, 200, rng)
    out = m.tracer_sample(Q, pts, [6])[:, 0]
    for x, v in zip(pts, out):
        p = m.find_leaf(x)
        h = m.geom[p, 3]
        u = (x[0] - m.geom[p, 0]) / h - 0.5
        t = u - np.floor(u)
        assert abs(v - (x[0] ** 2 + h * h * t * (1 - t))) < 1e-13


def test_samples_at_cell_centres_are_cell_values():
    m = amr_mesh()
    rng = np.random.default_rng(3)
    Q = rng.normal(size=m.zeros().shape)
    for p in (0, 3, m.np - 1):
        P = box_centers(m.geom[p, :3], m.geom[p, 3:])
        for idx in ((3, 3, 3), (7, 4, 11), (11, 11, 11)):
            x = P[idx]
            out = m.tracer_sample(Q, x[None, :], [0, 25, 58])
            np.testing.assert_allclose(out[0], Q[p][idx][[0, 25, 58]], rtol=0, atol=1e-14)


def test_points_outside_give_nan_and_do_not_move():
    m = amr_mesh()
    Q = m.zeros()
    pos = np.array([[0.1, 0.2, 0.0], [3.0, 0.0, 0.0]])
    out = m.tracer_sample(Q, pos, [7])
    assert np.isfinite(out[0, 0]) and np.isnan(out[1, 0])
    before = pos.copy()
    assert m.tracer_advance(Q, pos, 0.1) == 1
    assert np.array_equal(pos[1], before[1])


def test_euler_step_in_constant_and_linear_shift():
    """Puncture trackers move with -beta: x <- x - dt beta(x).  A constant shift moves every
    tracer by -dt beta; a linear shift beta = M x + b is interpolated exactly, so one step gives
    x - dt (M x + b)."""
    m = amr_mesh()
    rng = np.random.default_rng(4)
    M = rng.normal(size=(3, 3)) * 0.3
    b = rng.normal(size=3) * 0.1
    Q = m.zeros()
    for p in range(m.np):
        P = box_centers(m.geom[p, :3], m.geom[p, 3:])
        Q[p, ..., 7:10] = P @ M.T + b
    pos = interior_points(m, 50, rng) * 0.8
    x0 = pos.copy()
    dt = 0.05
    assert m.tracer_advance(Q, pos, dt) == 0
    np.testing.assert_allclose(pos, x0 - dt * (x0 @ M.T + b), rtol=0, atol=1e-14)
    Qc = m.zeros()
    Qc[..., 7:10] = b
    pos = x0.copy()
    m.tracer_advance(Qc, pos, dt)
    np.testing.assert_allclose(pos, x0 - dt * b, rtol=0, atol=1e-15)


def sphere_mesh(centres, radii):
    from paper_2406_11626_amd import scenarios
    n0, origin, extent = (4, 4, 2), (-2.0, -2.0, -1.0), (4.0, 4.0, 2.0)
    ref = scenarios.sphere_refinement(n0, origin, extent, centres, radii)
    return orc.Mesh(n0, origin, extent, 1, ref), ref


def test_tracker_tags_fixed_point_of_sphere_refinement():
    """A mesh refined by spheres of radii R_l around the tracers is left as it is."""
    centres = [(0.31, -0.12, 0.07), (-0.6, 0.5, -0.1)]
    radii = [0.9, 0.25]
    m, _ = sphere_mesh(centres, radii)
    assert m.ids[:, 0].max() == 2
    tags = m.tag_tracers(np.array(centres), radii, 2)
    assert np.all(tags == 0)


def test_tracker_tags_follow_a_moved_tracer():
    """Move the tracer: the plan of the tags reproduces the sphere refinement around the new
    position (the tag rule refines and coarsens exactly the cubes that differ)."""
    radii = [0.9, 0.25]
    m, _ = sphere_mesh([(0.31, -0.12, 0.07)], radii)
    new = (0.55, 0.1, 0.07)
    _, want = sphere_mesh([new], radii)
    cur = m
    for _ in range(3):  # refinement proceeds one level per regrid
        tags = cur.tag_tracers(np.array([new]), radii, 2)
        plan = cur.regrid_plan(tags, 2)
        cur = orc.Mesh((4, 4, 2), (-2.0, -2.0, -1.0), (4.0, 4.0, 2.0), 1, [tuple(c) for c in plan])
    assert {tuple(int(v) for v in c) for c in plan} == {tuple(c) for c in want}
    assert np.all(cur.tag_tracers(np.array([new]), radii, 2) == 0)


def test_tracker_tags_respect_max_level_and_far_leaves():
    """With the tracer moved more than R_0 + a cube diagonal away from every refined cube, every
    fine leaf is asked to coarsen and nothing near the tracer's old place refines."""
    radii = [0.3, 0.1]
    m, _ = sphere_mesh([(0.31, -0.12, 0.07)], radii)
    assert m.ids[:, 0].max() == 2
    far = np.array([[-1.95, 1.95, -0.95]])
    tags = m.tag_tracers(far, radii, 2)
    lev = m.ids[:, 0]
    assert np.all(tags[lev > 0] == -1)          # every fine leaf's parent is now far away
    t1 = m.tag_tracers(far, radii, 0)            # max_level 0: nothing is refined
    assert not np.any(t1 == 1)

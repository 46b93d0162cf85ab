"""GPU parity of tracers, puncture trackers and refinement tags by coordinates against the
oracle: trilinear samples at random points of a static AMR mesh (NaN outside), several Euler
steps of trackers in a random shift field, and the REFINE / KEEP / COARSEN tags around moved
tracers on a sphere-refined mesh (integers: bit-exact)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as orc  # noqa: E402
from gpu_helpers import to_gpu  # noqa: E402
from paper_2406_11626_amd import ccz4, scenarios  # noqa: E402
from seeded_inputs import box_centers, smooth_state  # noqa: E402

N0, ORIGIN, EXTENT = (3, 3, 2), (-1.5, -1.5, -1.0), (3.0, 3.0, 2.0)
REFINED = [(0, 1, 1, 0), (0, 1, 1, 1)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ccz4.lib()


def pair(refined=REFINED):
    ctx = ccz4.Context(N0, ORIGIN, EXTENT, ccz4.BC_NEUMANN, ccz4.params(), refined)
    m = orc.Mesh(N0, ORIGIN, EXTENT, ccz4.BC_NEUMANN, refined)
    assert np.array_equal(ctx.ids, m.ids)
    return ctx, m


def state(m, seed):
    Q = m.zeros()
    for p in range(m.np):
        Q[p] = smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), seed)
    m.fill_halos(Q)
    return Q


def points(n, seed, outside=0):
    rng = np.random.default_rng(seed)
    P = np.array(ORIGIN) + rng.random((n, 3)) * np.array(EXTENT) * 0.999
    if outside:
        P[:outside] += np.array([5.0, 0.0, 0.0])
    return P


def test_tracer_samples_match_oracle():
    ctx, m = pair()
    Qo = state(m, 70)
    pts = points(500, 1, outside=3)
    slots = [0, 6, 7, 10, 17, 25, 40, 57, 58]
    want = m.tracer_sample(Qo, pts, slots)
    got = ctx.tracers_sample(to_gpu(Qo), torch.tensor(pts, device="cuda"), slots).cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(want)) and np.isnan(got[:3]).all()
    ok = ~np.isnan(want)
    assert np.abs(got[ok] - want[ok]).max() <= 1e-13 * np.abs(want[ok]).max()


def test_tracer_samples_near_leaf_edges_match_oracle():
    """Points within half a cell of inner leaf edges and corners, on a mesh with refined leaves,
    interiors set to a multilinear field and every halo cell NaN before the fill (which writes
    face halos only): the eight cells come from the same-level leaves that hold them, so samples
    whose cells all have a same-level owner are exact, and the rest (next to coarse-fine edges)
    read the face halo, or NaN from an unwritten edge region, exactly as the oracle does."""
    ctx, m = pair()
    rng = np.random.default_rng(11)
    c = rng.normal(size=8)

    def f(x, y, z):
        return c[0] + c[1] * x + c[2] * y + c[3] * z + c[4] * x * y + c[5] * x * z + c[6] * y * z + c[7] * x * y * z

    Q = m.zeros()
    for p in range(m.np):
        P = box_centers(m.geom[p, :3], m.geom[p, 3:])
        Q[p, ..., 9] = f(P[..., 0], P[..., 1], P[..., 2])
    inner = np.zeros((15, 15, 15), bool)
    inner[3:12, 3:12, 3:12] = True
    Q[:, ~inner, :] = np.nan
    m.fill_halos(Q)
    pts = []
    h = 0.5 / 9  # half a level-0 cell
    for _ in range(200):  # near the inner level-0 edges (x, y in {-0.5, 0.5}, z = 0) and around them
        e = np.array([rng.choice([-0.5, 0.5]), rng.choice([-0.5, 0.5]), 0.0]) + rng.uniform(-h, h, 3) * 0.999
        e[rng.integers(0, 3)] = rng.uniform(-1.4, 1.4) if rng.random() < 0.5 else e[0]
        pts.append(e)
    pts = np.array(pts)
    want = m.tracer_sample(Q, pts, [9])
    got = ctx.tracers_sample(to_gpu(Q), torch.tensor(pts, device="cuda"), [9]).cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want[:, 0])
    assert ok.sum() > 100
    assert np.abs(got[ok, 0] - want[ok, 0]).max() <= 1e-13 * np.abs(want[ok, 0]).max()
    # where every cell has a level-0 owner the sample is the field itself
    lev0 = np.array([m.ids[m.find_leaf(x), 0] == 0 for x in pts])
    np.testing.assert_allclose(want[ok & lev0, 0], f(*pts[ok & lev0].T), rtol=0, atol=1e-12)


def test_tracer_points_within_rounding_of_faces_match_oracle():
    """Points on leaf faces and corners and within rounding of them (offsets down to subnormal)
    are found in a leaf exactly where the oracle finds one: both take the point's cube index at
    the finest level, so no point falls between two leaves."""
    ctx, m = pair()
    Qo = state(m, 72)
    rng = np.random.default_rng(5)
    corners = np.unique(np.concatenate([m.geom[:, :3], m.geom[:, :3] + 9 * m.geom[:, 3:]]), axis=0)
    pts = np.array([c + rng.choice([-1e-300, 0.0, 1e-300, -1e-17, 1e-17, -3e-26], size=3)
                    for c in corners for _ in range(3)])
    slots = [7, 8, 9, 17]
    want = m.tracer_sample(Qo, pts, slots)
    got = ctx.tracers_sample(to_gpu(Qo), torch.tensor(pts, device="cuda"), slots).cpu().numpy()
    assert np.array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    inner = np.all(pts > np.array(ORIGIN) + 1e-12, axis=1) & np.all(pts < np.array(ORIGIN) + np.array(EXTENT) - 1e-12,
                                                                     axis=1)
    assert ok[inner].all()  # every point inside the domain is in a leaf
    assert np.abs(got[ok] - want[ok]).max() <= 1e-13 * np.abs(want[ok]).max()


def test_tracker_euler_steps_match_oracle():
    ctx, m = pair()
    Qo = state(m, 71)
    Qd = to_gpu(Qo)
    pos = points(64, 2, outside=1) * 0.6
    pos[0] = [7.0, 0.0, 0.0]
    pd = torch.tensor(pos, device="cuda")
    for _ in range(5):
        m.tracer_advance(Qo, pos, 0.05)
        ctx.tracers_advance(Qd, pd, 0.05)
    got = pd.cpu().numpy()
    assert np.array_equal(got[0], [7.0, 0.0, 0.0])
    assert np.abs(got - pos).max() <= 1e-14 * max(1.0, np.abs(pos).max())


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tracker_tags_match_oracle(seed):
    radii = [0.8, 0.3]
    centres = [(0.2, -0.1, 0.05), (-0.4, 0.3, -0.2)]
    ref = scenarios.sphere_refinement(N0, ORIGIN, EXTENT, centres, radii)
    ctx, m = pair(ref)
    rng = np.random.default_rng(seed)
    moved = np.array(centres) + rng.normal(size=(2, 3)) * 0.3 * seed
    want = m.tag_tracers(moved, radii, 2)
    got = ctx.tag_tracers(torch.tensor(moved, device="cuda"), radii, 2).cpu().numpy()
    assert np.array_equal(got, want)
    if seed == 0:
        assert np.all(got == 0)  # the sphere refinement around the tracers is a fixed point
    else:
        assert (got == 1).any() or (got == -1).any()


def test_empty_tracer_set():
    """No tracers: sampling and advancing return at once and leave their buffers as they were, and
    the tags by coordinates of an empty set are the oracle's: no leaf lies near a tracer, so every
    leaf above the base level has its parent cube far from all of them (COARSEN) and the base
    level keeps (KEEP)."""
    radii = [0.8, 0.3]
    ref = scenarios.sphere_refinement(N0, ORIGIN, EXTENT, [(0.2, -0.1, 0.05)], radii)
    ctx, m = pair(ref)
    Q = ctx.new_state(0.0)
    pos = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    out = torch.full((1, 2), 7.0, dtype=torch.float64, device="cuda")
    ccz4.ccz4_tracers_sample(ctx.h, Q, pos, [0, 1], out)
    ccz4.ccz4_tracers_advance(ctx.h, Q, pos, 0.1)
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)
    want = m.tag_tracers(np.zeros((0, 3)), radii, 2)
    got = ctx.tag_tracers(pos, radii, 2).cpu().numpy()
    assert np.array_equal(got, want)
    lev = np.asarray(ctx.ids)[:, 0]
    assert (lev >= 1).any() and np.all(got[lev >= 1] == -1) and np.all(got[lev == 0] == 0)


def test_tracer_arguments_are_checked():
    ctx, _ = pair()
    Q = ctx.new_state(0.0)
    pos = torch.zeros((2, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(ccz4.CCZ4Error):
        ccz4.ccz4_tracers_sample(ctx.h, Q, pos, [59], torch.empty((2, 1), dtype=torch.float64, device="cuda"))
    with pytest.raises(ccz4.CCZ4Error):
        ccz4.ccz4_tag_tracers(ctx.h, pos, [0.1] * 17, 2, torch.empty(ctx.n_patches, dtype=torch.int8, device="cuda"))

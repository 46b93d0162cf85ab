"""GPU parity of the second-order formulation against the oracle: the right-hand side without
the red terms (auxiliaries' right-hand sides zero), the FD4 reconstruction of A, B, D, P with
and without the same-level halo push, and whole fused RK4 steps (Algorithm 2 with RK4) on the
gauge wave, the puncture with Sommerfeld ghosts and a static AMR mesh, eager and as a graph.
Same 1e-12 normwise measure per slot as the first-order parity tests."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as orc  # noqa: E402
from gpu_helpers import (INTERIOR, SLABS, oracle_sensitivity, parity_error, same_level_halo_mask,  # noqa: E402
                         sensitivity, to_gpu, to_host, ulp_perturbed)
from paper_2406_11626_amd import ccz4, scenarios  # noqa: E402
from seeded_inputs import box_centers, smooth_state  # noqa: E402

KERNELS = [ccz4.KERNEL_PHASED, ccz4.KERNEL_LDS]
AUX = slice(25, 58)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ccz4.lib()


def so_params(w=None, **kw):
    base = dict(w.prm) if w is not None else {}
    base.update(kw)
    base["formulation"] = ccz4.FORMULATION_SO
    return ccz4.params(**base)


def oparams(prm):
    return orc.Params(**{f: getattr(prm, f) for f, _ in ccz4.Params._fields_})


def make_pair(n0, origin, extent, bc, prm, refined=(), kernel=ccz4.KERNEL_LDS):
    ctx = ccz4.Context(n0, origin, extent, bc, prm, refined)
    for prec in (ccz4.PREC_FP64, ccz4.PREC_MIXED):
        ctx.set_kernel(prec, kernel)
    m = orc.Mesh(n0, origin, extent, bc, refined)
    assert np.array_equal(ctx.ids, m.ids)
    return ctx, m


def random_state(m, seed, frozen=False):
    Q = m.zeros()
    for p in range(m.np):
        Q[p] = smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), seed, frozen_shift=frozen)
    return Q


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("shift", [1, 0])
def test_so_rhs_parity_random_states(kernel, shift):
    prm = so_params(slicing=shift, shift=shift, kappa1=0.3, kappa3=0.5 * shift)
    ctx, m = make_pair((2, 2, 1), (-0.4, 0.1, 0.2), (1.6, 1.6, 0.8), ccz4.BC_PERIODIC, prm, kernel=kernel)
    Qo = random_state(m, 40 + shift, frozen=shift == 0)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    kd = ctx.new_state(1.0)
    ctx.rhs(Qd, kd)
    ko = m.rhs(oparams(prm), Qo)
    g = to_host(kd)
    e = parity_error(g, ko)
    assert e.max() <= 1e-12, (e.argmax(), e.max())
    assert np.all(g[:, 3:12, 3:12, 3:12, AUX] == 0.0)
    # the first-order right-hand side of the same state differs in Ghat and b only among the
    # primaries (the red terms)
    ctx_fo = ccz4.Context((2, 2, 1), (-0.4, 0.1, 0.2), (1.6, 1.6, 0.8), ccz4.BC_PERIODIC,
                          ccz4.params(**{f: getattr(prm, f) for f, _ in ccz4.Params._fields_ if f != "formulation"}))
    ctx_fo.set_kernel(ccz4.PREC_FP64, kernel)
    kf = ctx_fo.new_state(0.0)
    ctx_fo.rhs(Qd, kf)
    f = to_host(kf)[:, 3:12, 3:12, 3:12]
    same = list(range(0, 19))
    np.testing.assert_array_equal(f[..., same], g[:, 3:12, 3:12, 3:12][..., same])


@pytest.mark.parametrize("push", [False, True])
def test_reconstruct_parity_and_push(push):
    """Interior auxiliaries against the oracle's reconstruction; primaries untouched; with push,
    the auxiliaries' face halos on a periodic mesh (all faces same-level) equal those of the
    oracle's fill after its reconstruction, bit for bit."""
    prm = so_params()
    ctx, m = make_pair((3, 2, 2), (-0.4, 0.1, 0.2), (2.4, 1.6, 1.6), ccz4.BC_PERIODIC, prm)
    Qo = random_state(m, 51)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    ctx.reconstruct(Qd, push=push)
    Ro = Qo.copy()
    m.reconstruct(Ro)
    g = to_host(Qd)
    e = parity_error(g, Ro)
    assert e.max() <= 1e-12, (e.argmax(), e.max())
    np.testing.assert_array_equal(g[..., :25], Qo[..., :25])
    np.testing.assert_array_equal(g[..., 58], Qo[..., 58])
    if push:
        # the pushed halo values are copies of the neighbours' new interior values: a plain
        # same-level fill of the result changes nothing
        Hd = to_gpu(g)
        ctx.fill_halos(Hd)
        H = to_host(Hd)
        np.testing.assert_array_equal(np.where(SLABS[..., None], g, 0.0), np.where(SLABS[..., None], H, 0.0))
        assert not np.array_equal(np.where(SLABS[..., None], g, 0.0)[..., AUX],
                                  np.where(SLABS[..., None], Qo, 0.0)[..., AUX])
    else:
        # no halo is written
        np.testing.assert_array_equal(np.where(SLABS[..., None], g, 0.0), np.where(SLABS[..., None], Qo, 0.0))


@pytest.mark.parametrize("periodic", [True, False])
def test_reconstruct_gather_reads_same_level_halos_from_the_neighbours(periodic):
    """With CCZ4_STAGE_GATHER_SAME_LEVEL the reconstruction reads the primaries' same-level y and z
    face halos from the neighbours' interiors: with those halos overwritten by NaN it writes the
    same auxiliaries (interior and pushed halos, with no push, the x-face push and the full push)
    as on the filled state, on a periodic mesh and on one with coarse-fine and Sommerfeld faces."""
    if periodic:
        ctx, m = make_pair((3, 2, 2), (-0.4, 0.1, 0.2), (2.4, 1.6, 1.6), ccz4.BC_PERIODIC, so_params())
        Qo = random_state(m, 53)
        m.fill_halos(Qo)
        Q = to_gpu(Qo)
    else:
        w = scenarios.config(2)
        ctx = ccz4.Context((3, 3, 2), (-9.0, -9.0, -6.0), (18.0, 18.0, 12.0), w.bc, so_params(w), [(0, 1, 1, 0)])
        Q = ctx.new_state(0.0)
        ctx.init_patches(Q, w.scenario, w.scen)
        ctx.fill_halos(Q)
    prim = torch.zeros_like(Q, dtype=torch.bool)
    prim[:, :11] = True
    mask = same_level_halo_mask(ctx, Q, axes=(1, 2)) & prim
    assert int(mask.sum()) > 0
    G = Q.clone()
    G[mask] = float("nan")
    for fl in (0, ccz4.STAGE_FILL_SAME_LEVEL_X, ccz4.STAGE_FILL_SAME_LEVEL):
        R, H = Q.clone(), G.clone()
        ctx.reconstruct(R, flags=fl)
        ctx.reconstruct(H, flags=fl | ccz4.STAGE_GATHER_SAME_LEVEL)
        assert bool(torch.isfinite(H[~mask]).all()), fl
        assert torch.equal(H[~mask], R[~mask]), (fl, int((H[~mask] != R[~mask]).sum()))
    with pytest.raises(ccz4.CCZ4Error):
        ccz4.ccz4_reconstruct_aux(ctx.h, Q, 8)


def _so_steps(w, n0, prm, refined=(), steps=2, perturb=False, kernel=ccz4.KERNEL_LDS, push=True, graph=False):
    ctx, m = make_pair(n0, w.origin, w.extent, w.bc, prm, refined, kernel=kernel)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    if perturb:
        for p in range(m.np):
            Qo[p, 3:12, 3:12, 3:12] += 1e-3 * smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), 52)[3:12, 3:12, 3:12]
    m.set_background(Qo)
    m.fill_halos(Qo)
    m.reconstruct(Qo)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    ctx.set_background(to_gpu(Qo))
    bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    pr = oparams(prm)
    dt = w.dt()
    sg = ccz4.StepGraph(ctx, Qd, bufs, dt) if graph else None

    def run(Q):
        for _ in range(steps):
            Q = m.rk4_step(pr, Q, dt)
        return Q
    for _ in range(steps):
        if sg is not None:
            sg.launch()
        else:
            ctx.rk4_step_fused(Qd, dt, bufs, push=push)
    torch.cuda.synchronize()
    if sg is not None:
        sg.close()
    Q0 = Qo
    Qo = run(Q0.copy())
    # the oracle's own sensitivity to one-ulp changes of the initial state (gpu_helpers.KAPPA)
    sens = oracle_sensitivity(run, Q0, ref=Qo)
    return ctx, m, to_host(Qd), Qo, sens


@pytest.mark.parametrize("push", [True, False])
@pytest.mark.parametrize("kernel", KERNELS)
def test_so_fused_steps_gauge_wave_match_oracle(kernel, push):
    w = scenarios.config(1)
    _, _, g, Qo, sens = _so_steps(w, w.n0, so_params(w), steps=6, kernel=kernel, push=push)
    e = parity_error(g, Qo, sens=sens, tol=1e-11)
    assert e.max() <= 1e-11, (e.argmax(), e.max())


@pytest.mark.parametrize("kernel", KERNELS)
def test_so_fused_steps_puncture_sommerfeld_match_oracle(kernel):
    w = scenarios.config(2)
    _, m, g, Qo, sens = _so_steps(w, (2, 2, 2), so_params(w), steps=2, perturb=True, kernel=kernel)
    e = parity_error(g, Qo, sens=sens, tol=1e-11)
    assert e.max() <= 1e-11, (e.argmax(), e.max())


def test_so_fused_steps_static_amr_match_oracle():
    """Coarse-fine faces: the reconstruction's auxiliaries reach fine and coarse halos through
    restriction and prolongation after each stage."""
    w = scenarios.config(2)
    refined = [(0, 1, 1, 1)]
    _, m, g, Qo, sens = _so_steps(w, (3, 3, 3), so_params(w), refined=refined, steps=2, perturb=True)
    e = parity_error(g, Qo, sens=sens, tol=1e-11)
    assert e.max() <= 1e-11, (e.argmax(), e.max())


def test_so_step_graph_matches_oracle():
    w = scenarios.config(2)
    _, _, g, Qo, sens = _so_steps(w, (2, 2, 2), so_params(w), steps=2, perturb=True, graph=True)
    e = parity_error(g, Qo, sens=sens, tol=1e-11)
    assert e.max() <= 1e-11, (e.argmax(), e.max())


def test_full_size_so_step_graph_config4_sampled():
    """The second-order formulation on the full 24^3-leaf puncture mesh, one captured RK4 step
    (with its reconstructions) in the benchmark's launch configuration, against the oracle on
    sampled leaves.  Each sampled leaf is stepped on an oracle sub-box of the leaves within three
    of it: per stage the stencils reach 3 cells and the reconstruction 2 more, so one step and the
    initial reconstruction reach 22 cells, less than the 27 of three leaves.  The sub-boxes'
    initial data (bit-identical geometry) are uploaded into the GPU state before the
    reconstruction, so that both sides start from the same values wherever the step can look."""
    w = scenarios.config(4)
    prm = so_params(w)
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, prm, w.refined)
    index = {tuple(r[1:]): p for p, r in enumerate(ctx.ids)}
    samples = [(0, 0, 0), (0, 12, 23), (12, 12, 12)]  # a corner, a boundary face and edge, the puncture
    L = w.extent[0] / w.n0[0]
    Qd = ctx.new_state(0.0)
    ctx.init_patches(Qd, w.scenario, w.scen)
    subs = []
    for ijk in samples:
        lo = [max(0, c - 3) for c in ijk]
        n = [min(w.n0[a] - 1, ijk[a] + 3) - lo[a] + 1 for a in range(3)]
        m = orc.Mesh(tuple(n), tuple(w.origin[a] + lo[a] * L for a in range(3)), tuple(n[a] * L for a in range(3)), w.bc)
        Q = m.zeros()
        m.init(Q, w.scenario, w.scen)
        full = [index[(r[1] + lo[0], r[2] + lo[1], r[3] + lo[2])] for r in m.ids]
        np.testing.assert_array_equal(ctx.geom[full], m.geom)
        Qd[torch.tensor(full, device="cuda")] = to_gpu(Q)
        here = [q for q, r in enumerate(m.ids) if (r[1] + lo[0], r[2] + lo[1], r[3] + lo[2]) == ijk][0]
        subs.append((m, Q, here, index[ijk]))
    ctx.set_background(Qd)
    ctx.fill_halos(Qd)
    ctx.reconstruct(Qd, True)
    ctx.fill_halos(Qd)
    ctx.autotune(Qd, reps=1)
    ctx.fill_halos(Qd)
    dt = w.dt()
    bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    g = ctx.step_graph(Qd, bufs, dt)
    g.launch()
    torch.cuda.synchronize()
    g.close()
    del bufs
    got = to_host(Qd, [s_[3] for s_ in subs])
    del Qd
    torch.cuda.empty_cache()
    pr = oparams(prm)
    for k, (m, Q, here, _) in enumerate(subs):
        m.set_background(Q)
        m.fill_halos(Q)
        m.reconstruct(Q)
        m.fill_halos(Q)

        def run(Q0, m=m):
            return m.rk4_step(pr, Q0, dt)
        ref = run(Q.copy())
        r1, g1 = ref[here:here + 1], got[k:k + 1]
        e = parity_error(g1, r1)
        if e.max() > 1e-11:  # a cancellation residual: the oracle's own one-ulp sensitivity decides
            runs = [run(np.where(Q == 0.0, Q, ulp_perturbed(Q, 1234 + t))) for t in range(2)]
            e = parity_error(g1, r1, sens=sensitivity(r1, [r_[here:here + 1] for r_ in runs]), tol=1e-11)
        assert e.max() <= 1e-11, (samples[k], e.argmax(), e.max())
        assert np.abs(r1[:, 3:12, 3:12, 3:12] - Q[here:here + 1, 3:12, 3:12, 3:12]).max() > 1e-10


def test_reconstruct_rejects_bad_arguments():
    ctx = ccz4.Context((1, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), ccz4.BC_PERIODIC, so_params())
    Q = ctx.new_state(0.0)
    with pytest.raises(ccz4.CCZ4Error):
        ccz4.ccz4_reconstruct_aux(ctx.h, Q, 8)
    with pytest.raises(ccz4.CCZ4Error):
        ccz4.ccz4_reconstruct_aux(ctx.h, None, 0)

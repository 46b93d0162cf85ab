"""GPU parity: every C-ABI call of the hot path against the CPU oracle on the same seeded
inputs.  Floating-point results must agree to 1e-12 per slot in the normwise measure of
gpu_helpers.parity_error; pure copies must agree bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as orc  # noqa: E402
from gpu_helpers import (FLOOR, INTERIOR, SLABS, oracle_sensitivity, parity_error, perturbed_runs,  # noqa: E402
                         same_level_halo_mask, sensitivity, to_gpu, to_host, ulp_perturbed)
from paper_2406_11626_amd import ccz4, scenarios  # noqa: E402
from seeded_inputs import box_centers, smooth_state  # noqa: E402

TOL = 1e-12
KERNELS = [ccz4.KERNEL_PHASED, ccz4.KERNEL_LDS]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ccz4.lib()


def oparams(prm):
    return orc.Params(**{f: getattr(prm, f) for f, _ in ccz4.Params._fields_})


def make_pair(n0, origin, extent, bc, prm, refined=(), kernel=ccz4.KERNEL_LDS):
    ctx = ccz4.Context(n0, origin, extent, bc, prm, refined)
    for prec in (ccz4.PREC_FP64, ccz4.PREC_MIXED):
        ctx.set_kernel(prec, kernel)
        assert ctx.get_kernel(prec) == kernel
    m = orc.Mesh(n0, origin, extent, bc, refined)
    assert ctx.n_patches == m.np
    assert np.array_equal(ctx.ids, m.ids)
    np.testing.assert_allclose(ctx.geom, m.geom, rtol=1e-15, atol=1e-15)
    return ctx, m


def random_state(m, seed, frozen=False):
    Q = m.zeros()
    for p in range(m.np):
        Q[p] = smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), seed, frozen_shift=frozen)
    return Q


def acc_slot_error(a, b):
    """Per-slot relative difference of two fused-stage accumulators (device tensors, compared in
    their own private layout, every element of every patch)."""
    x = a.detach().cpu().numpy().reshape(a.shape[0], 59, -1)
    y = b.detach().cpu().numpy().reshape(b.shape[0], 59, -1)
    diff = np.abs(x - y).max(axis=(0, 2))
    scale = np.abs(y).max(axis=(0, 2))
    top = max(scale.max(), 1e-300)
    return diff / np.where(scale > FLOOR * top, scale, top)


def valid_accumulator(ctx, Q, dt=0.01):
    """An accumulator as stage 0 leaves it (Q + dt/6 RHS(Q) in the accumulator's own layout), so
    that a later stage, and the projection at s = 3, start from well-conditioned values."""
    acc, scratch = ctx.new_state(0.0), ctx.new_state(0.0)
    ctx.rhs_rk4_stage(0, dt, Q, Q, acc, scratch, ccz4.PREC_FP64, 0)
    return acc


# ------------------------------------------------------------------ initial data

@pytest.mark.parametrize("cfg", [1, 2, 5])
def test_init_parity(cfg):
    w = scenarios.config(cfg)
    n0 = (3, 3, 3) if cfg == 1 else (2, 2, 2)
    ctx, m = make_pair(n0, w.origin, w.extent, w.bc, w.params())
    Qd = ctx.new_state(0.0)
    ctx.init_patches(Qd, w.scenario, w.scen)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    mask = INTERIOR | (SLABS if w.bc == ccz4.BC_SOMMERFELD else False)
    g = to_host(Qd)
    diff = np.abs(g - Qo)[:, mask].max()
    scale = np.abs(Qo).max()
    assert diff <= 1e-13 * scale, diff


# ------------------------------------------------------------------ halo fill

def test_fill_periodic_and_neumann_bitwise():
    for bc in (ccz4.BC_PERIODIC, ccz4.BC_NEUMANN):
        ctx, m = make_pair((3, 2, 2), (0, 0, 0), (3.0, 2.0, 2.0), bc, ccz4.params())
        Qo = random_state(m, 11)
        Qo[:, SLABS] = 0.0
        Qd = to_gpu(Qo)
        ctx.fill_halos(Qd)
        m.fill_halos(Qo)
        g = to_host(Qd)
        assert np.array_equal(g[:, SLABS], Qo[:, SLABS])
        assert np.array_equal(g[:, INTERIOR], Qo[:, INTERIOR])


def test_fill_single_patch_periodic_self_neighbour():
    ctx, m = make_pair((1, 1, 1), (0, 0, 0), (1.0, 1.0, 1.0), ccz4.BC_PERIODIC, ccz4.params())
    Qo = random_state(m, 12)
    Qd = to_gpu(Qo)
    ctx.fill_halos(Qd)
    m.fill_halos(Qo)
    assert np.array_equal(to_host(Qd)[:, SLABS], Qo[:, SLABS])


@pytest.mark.parametrize("bc", [ccz4.BC_PERIODIC, ccz4.BC_NEUMANN])
def test_fill_amr_restrict_prolong(bc):
    """Refined centre cube plus one second-level refinement: copy, restriction and
    prolongation faces of every orientation."""
    refined = [(0, 1, 1, 1), (1, 4, 4, 4)]
    ctx, m = make_pair((3, 3, 3), (0, 0, 0), (3.0, 3.0, 3.0), bc, ccz4.params(), refined)
    Qo = random_state(m, 13)
    Qo[:, SLABS] = 0.0
    Qd = to_gpu(Qo)
    ctx.fill_halos(Qd)
    m.fill_halos(Qo)
    e = parity_error(to_host(Qd), Qo, SLABS)
    assert e.max() <= 1e-14, e.max()


def test_fill_rejects_level_jumps():
    with pytest.raises(ccz4.CCZ4Error) as ei:
        ccz4.Context((3, 3, 3), (0, 0, 0), (3.0, 3.0, 3.0), ccz4.BC_PERIODIC, ccz4.params(),
                     [(0, 1, 1, 1), (1, 3, 4, 4)])
    assert ei.value.status == ccz4.CCZ4_ELAYOUT


# ------------------------------------------------------------------ right-hand side

PARAM_SETS = [
    dict(slicing=1, shift=1),
    dict(slicing=0, shift=0, kappa1=1.0, kappa3=0.0),
    dict(slicing=1, shift=1, kappa1=0.3, kappa2=0.4, kappa3=0.7, tau=0.7, e=1.5, c=0.8, mu=0.37, f=0.6, eta=1.3,
         ko_eps=0.8),
]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("ps", range(len(PARAM_SETS)))
def test_rhs_parity_random_states(ps, kernel):
    prm = ccz4.params(**PARAM_SETS[ps])
    ctx, m = make_pair((2, 2, 1), (-0.4, 0.1, 0.2), (1.6, 1.6, 0.8), ccz4.BC_PERIODIC, prm, kernel=kernel)
    Qo = random_state(m, 20 + ps, frozen=PARAM_SETS[ps]["shift"] == 0)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    kd = ctx.new_state(0.0)
    ctx.rhs(Qd, kd)
    ko = m.rhs(oparams(prm), Qo)
    e = parity_error(to_host(kd), ko)
    assert e.max() <= TOL, (e.argmax(), e.max())
    assert np.array_equal(to_host(Qd), Qo)  # Q untouched


@pytest.mark.parametrize("kernel", KERNELS)
def test_rhs_parity_gauge_wave_config1(kernel):
    w = scenarios.config(1)
    ctx, m = make_pair(w.n0, w.origin, w.extent, w.bc, w.params(), kernel=kernel)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    kd = ctx.new_state(0.0)
    ctx.rhs(Qd, kd)
    pr = oparams(w.params())
    ko = m.rhs(pr, Qo)
    # Theta's right-hand side on the exact gauge wave is a cancellation residual (7.5e-6 of the
    # largest slot): the oracle itself moves it by 2e-10 of its size under one-ulp input changes
    sens = oracle_sensitivity(lambda Q: m.rhs(pr, Q), Qo, ref=ko)
    e = parity_error(to_host(kd), ko, sens=sens, tol=TOL)
    assert e.max() <= TOL, (e.argmax(), e.max())


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("cfg", [2, 5])
def test_rhs_parity_punctures_with_sommerfeld_ghosts(cfg, kernel):
    w = scenarios.config(cfg)
    ctx, m = make_pair((2, 2, 2), w.origin, w.extent, w.bc, w.params(), kernel=kernel)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    ctx.set_background(Qd)
    kd = ctx.new_state(0.0)
    ctx.rhs(Qd, kd)
    ko = m.rhs(oparams(w.params()), Qo)
    g = to_host(kd)
    e = parity_error(g, ko, INTERIOR)
    assert e.max() <= TOL, (e.argmax(), e.max())
    e = parity_error(g, ko, SLABS)
    assert e.max() <= TOL, (e.argmax(), e.max())


# ------------------------------------------------------------------ RK4 stage

def test_rk4_stage_parity():
    ctx, m = make_pair((2, 1, 1), (-1, -1, -1), (2.0, 1.0, 1.0), ccz4.BC_SOMMERFELD, ccz4.params())
    Qn = random_state(m, 30)
    m.set_background(Qn)
    rng = np.random.default_rng(31)
    ks = [rng.normal(size=Qn.shape) for _ in range(4)]
    acc_o, Qx_o = m.zeros(), m.zeros()
    Qn_d = to_gpu(Qn)
    acc_d, Qx_d = ctx.new_state(0.0), ctx.new_state(0.0)
    ctx.set_background(Qn_d)
    dt = 0.013
    mask = INTERIOR | SLABS
    for s in range(4):
        m.rk4_stage(s, dt, Qn, ks[s], acc_o, Qx_o)
        ctx.rk4_stage(s, dt, Qn_d, to_gpu(ks[s]), acc_d, Qx_d)
        e = parity_error(to_host(Qx_d), Qx_o, mask)
        assert e.max() <= 1e-14, (s, e.argmax(), e.max())
        if s < 3:
            e = parity_error(to_host(acc_d), acc_o, mask)
            assert e.max() <= 1e-15, (s, e.max())
    with pytest.raises(ccz4.CCZ4Error):
        ctx.rk4_stage(4, dt, Qn_d, Qn_d, acc_d, Qx_d)
    with pytest.raises(ccz4.CCZ4Error):
        ctx.rk4_stage(0, 0.0, Qn_d, Qn_d, acc_d, Qx_d)


# ------------------------------------------------------------------ constraints and tags

def test_constraints_parity_and_norms():
    w = scenarios.config(5)
    ctx, m = make_pair((2, 2, 2), w.origin, w.extent, w.bc, w.params())
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    HMd = torch.zeros((ctx.n_patches, 4, 729), dtype=torch.float64, device="cuda")
    norms_d, st = ctx.constraints(Qd, HMd, r_excise=0.5)
    assert st == ccz4.CCZ4_OK
    norms_o, HMo = m.constraints(Qo, r_excise=0.5, want_fields=True)
    g = HMd.cpu().numpy().transpose(0, 2, 1)
    for q in range(4):
        scale = np.abs(HMo[..., q]).max()
        assert np.abs(g[..., q] - HMo[..., q]).max() <= TOL * scale
    np.testing.assert_allclose(norms_d[:2], norms_o[:2], rtol=1e-12)
    assert norms_d[2] == norms_o[2] == 0
    # one non-finite value is counted and reported
    Qd[1, 17, 5, 6, 7] = float("nan")
    norms_d, st = ctx.constraints(Qd)
    assert st == ccz4.CCZ4_ENONFINITE and norms_d[2] >= 1


def test_full_size_constraints_config4_sampled():
    """The constraint monitor's launch over the full 24^3-leaf puncture (13,824 leaves): H and M_i
    of sampled leaves against the oracle on sub-boxes of the leaves around each (the sub-boxes'
    initial data uploaded into the GPU state, so that both sides read the same values), each
    quantity measured against its largest magnitude over the mesh, as the small-mesh test measures
    it over its whole mesh.  Samples: a domain corner, the two leaves that meet at the puncture
    diagonally, an interior leaf."""
    w = scenarios.config(4)
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, w.params(), w.refined)
    index = {tuple(r[1:]): p for p, r in enumerate(ctx.ids)}
    Qd = ctx.new_state(0.0)
    ctx.init_patches(Qd, w.scenario, w.scen)
    samples = [(0, 0, 0), (11, 11, 11), (12, 12, 12), (5, 17, 9)]
    subs = []
    for ijk in samples:
        m, lo, Q = _subbox_oracle(w, ijk, margin=1)
        full = [index[(r[1] + lo[0], r[2] + lo[1], r[3] + lo[2])] for r in m.ids]
        Qd[torch.tensor(full, device="cuda")] = to_gpu(Q)
        here = [p for p, r in enumerate(m.ids) if (r[1] + lo[0], r[2] + lo[1], r[3] + lo[2]) == ijk][0]
        subs.append((m, Q, here))
    ctx.fill_halos(Qd)
    HMd = torch.zeros((ctx.n_patches, 4, 729), dtype=torch.float64, device="cuda")
    norms, st = ctx.constraints(Qd, HMd)
    assert st == ccz4.CCZ4_OK and norms[2] == 0
    scale = HMd.abs().amax(dim=(0, 2)).cpu().numpy()
    g = HMd[torch.tensor([index[ijk] for ijk in samples], device="cuda")].cpu().numpy().transpose(0, 2, 1)
    del Qd, HMd
    torch.cuda.empty_cache()
    for n, (m, Q, here) in enumerate(subs):
        m.fill_halos(Q)
        _, HMo = m.constraints(Q, want_fields=True)
        d = np.abs(g[n] - HMo[here]).max(0)
        assert (d <= TOL * scale).all(), (samples[n], d / scale)
        assert np.abs(HMo[here]).max() > 0


def test_tag_refine_parity():
    w = scenarios.config(2)
    refined = [(0, 0, 0, 0)]
    ctx, m = make_pair((2, 2, 2), w.origin, w.extent, ccz4.BC_NEUMANN, w.params(), refined)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    ind_o = m.tag_indicator(Qo)
    ind_d = torch.zeros((ctx.n_patches, 3), dtype=torch.float64, device="cuda")
    tags_d = torch.zeros(ctx.n_patches, dtype=torch.int8, device="cuda")
    emax = ind_o.max(1)
    theta_r = float(np.quantile(emax, 0.7))
    theta_c = float(np.quantile(emax, 0.3))
    ctx.tag_refine(Qd, theta_r, theta_c, 2, tags_d, ind_d)
    np.testing.assert_allclose(ind_d.cpu().numpy(), ind_o, rtol=1e-12, atol=1e-300)
    tags_o = m.tag_refine(Qo, theta_r, theta_c, 2)
    near = (np.abs(emax - theta_r) < 1e-12 * theta_r) | (np.abs(emax - theta_c) < 1e-12 * theta_c)
    t = tags_d.cpu().numpy()
    assert np.array_equal(t[~near], tags_o[~near])
    assert set(np.unique(t)) <= {-1, 0, 1}


def test_full_size_tag_refine_config4_sampled():
    """The plain refinement criterion over the full 24^3-leaf puncture: the indicator (largest
    adjacent differences of chi and alpha, dx^2 max|H|) of sampled leaves against the oracle on
    sub-boxes of the leaves around each (initial data uploaded as in the other full-size tests)
    at 1e-12 of each indicator's size on the mesh, and their tags with thresholds at the 99th and 30th percentiles of the mesh's
    indicator (level-0 leaves: REFINE or KEEP).  Samples: a domain corner, the two leaves at the
    puncture, an interior leaf."""
    w = scenarios.config(4)
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, w.params(), w.refined)
    index = {tuple(r[1:]): p for p, r in enumerate(ctx.ids)}
    Qd = ctx.new_state(0.0)
    ctx.init_patches(Qd, w.scenario, w.scen)
    samples = [(0, 0, 0), (11, 11, 11), (12, 12, 12), (5, 17, 9)]
    subs = []
    for ijk in samples:
        m, lo, Q = _subbox_oracle(w, ijk, margin=1)
        full = [index[(r[1] + lo[0], r[2] + lo[1], r[3] + lo[2])] for r in m.ids]
        Qd[torch.tensor(full, device="cuda")] = to_gpu(Q)
        here = [p for p, r in enumerate(m.ids) if (r[1] + lo[0], r[2] + lo[1], r[3] + lo[2]) == ijk][0]
        subs.append((m, Q, here))
    ctx.fill_halos(Qd)
    ind_d = torch.zeros((ctx.n_patches, 3), dtype=torch.float64, device="cuda")
    tags_d = torch.zeros(ctx.n_patches, dtype=torch.int8, device="cuda")
    ctx.tag_refine(Qd, 1e300, 0.0, 1, tags_d, ind_d)  # first pass: the indicator only
    emax = ind_d.max(1).values.cpu().numpy()
    theta_r, theta_c = float(np.quantile(emax, 0.99)), float(np.quantile(emax, 0.3))
    ctx.tag_refine(Qd, theta_r, theta_c, 1, tags_d, ind_d)
    sel = torch.tensor([index[ijk] for ijk in samples], device="cuda")
    ind_g, tags_g = ind_d[sel].cpu().numpy(), tags_d[sel].cpu().numpy()
    ind_scale = ind_d.amax(0).cpu().numpy()  # each indicator's largest value over the mesh
    t_all = tags_d.cpu().numpy()
    del Qd
    torch.cuda.empty_cache()
    assert (t_all == 1).sum() > 0 and set(np.unique(t_all)) <= {0, 1}
    for n, (m, Q, here) in enumerate(subs):
        m.fill_halos(Q)
        ind_o = m.tag_indicator(Q)[here]
        # each indicator to 1e-12 of its size on the mesh (the constraint term of a far-field leaf is
        # the truncation residual of H, 1e-10 of its size at the puncture, and rounds accordingly)
        assert (np.abs(ind_g[n] - ind_o) <= 1e-12 * ind_scale).all(), (samples[n], ind_g[n], ind_o)
        e = ind_o.max()
        if abs(e - theta_r) > 1e-12 * theta_r:  # ties decided in the same precision: none expected here
            assert tags_g[n] == (1 if e >= theta_r else 0), (samples[n], e, theta_r, tags_g[n])
    assert tags_g[2] == 1  # the leaf at the puncture refines


# ------------------------------------------------------------------ whole steps

def test_config1_ten_rk4_steps_match_oracle():
    w = scenarios.config(1)
    ctx, m = make_pair(w.n0, w.origin, w.extent, w.bc, w.params())
    Qd = ctx.new_state(0.0)
    ctx.init_patches(Qd, w.scenario, w.scen)
    Q0 = m.zeros()
    m.init(Q0, w.scenario, w.scen)
    bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    pr = oparams(w.params())

    def run(Q):
        for _ in range(w.steps):
            Q = m.rk4_step(pr, Q, w.dt())
        return Q
    for _ in range(w.steps):
        ctx.rk4_step(Qd, w.dt(), bufs)
    Qo = run(Q0.copy())
    sens = oracle_sensitivity(run, Q0, ref=Qo)
    e = parity_error(to_host(Qd), Qo, sens=sens, tol=1e-11)
    assert e.max() <= 1e-11, (e.argmax(), e.max())


# ------------------------------------------------------------------ full-size workloads, sampled

def _sample_patches(ids, n=24, seed=0):
    rng = np.random.default_rng(seed)
    lev = ids[:, 0]
    pick = set(rng.choice(len(ids), size=min(n, len(ids)), replace=False).tolist())
    pick.update([0, len(ids) - 1])
    for L in np.unique(lev):
        pick.add(int(np.where(lev == L)[0][0]))
        pick.add(int(np.where(lev == L)[0][-1]))
    return sorted(pick)


@pytest.mark.parametrize("cfg", [2, 3])
def test_full_size_sampled(cfg):
    """The whole configuration-2/3 mesh in the launch configuration of the benchmark.
    (a) RHS: the oracle-initialised, oracle-filled state is uploaded and the GPU RHS of sampled
    leaves (every level, domain corners, coarse-fine faces) is compared with the oracle's;
    (b) init: the GPU initial data of those leaves against the oracle's;
    (c) fill: the GPU fill of the uploaded interiors against the oracle's halos."""
    w = scenarios.config(cfg)
    ctx, m = make_pair(w.n0, w.origin, w.extent, w.bc, w.params(), w.refined)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    m.fill_halos(Qo)
    sel = _sample_patches(m.ids)
    # the exact data are constraint satisfying, so slots such as Theta (whose right-hand side
    # is then alpha R / 2, a truncation-error residual of large Ricci terms) carry no
    # significant digits to compare: perturb the sampled boxes by a smooth seeded field
    Qr = Qo[sel].copy()
    for n, p in enumerate(sel):
        Qr[n] += 1e-3 * smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), 40 + n)
    Qfull = Qo.copy()
    Qfull[sel] = Qr
    ko = m.rhs(oparams(w.params()), Qfull, k=np.zeros_like(Qo), subset=sel)[sel]
    del Qfull
    Qd = to_gpu(Qo)
    ctx.set_background(Qd)  # the unperturbed initial data, as on the oracle side
    Qd[torch.tensor(sel, device="cuda")] = to_gpu(Qr)
    del Qr
    kd = ctx.new_state(0.0)
    ctx.rhs(Qd, kd)
    e = parity_error(to_host(kd, sel), ko, INTERIOR)
    assert e.max() <= TOL, ("rhs", e.argmax(), e.max())
    if w.bc == ccz4.BC_SOMMERFELD:
        e = parity_error(to_host(kd, sel), ko, SLABS)
        assert e.max() <= TOL, ("rhs ghosts", e.argmax(), e.max())
    # the other kernel on the same full mesh
    ctx.set_kernel(ccz4.PREC_FP64, ccz4.KERNEL_PHASED)
    ctx.rhs(Qd, kd)
    e = parity_error(to_host(kd, sel), ko, INTERIOR)
    assert e.max() <= TOL, ("rhs phased", e.argmax(), e.max())
    ctx.set_kernel(ccz4.PREC_FP64, ccz4.KERNEL_LDS)
    del kd
    # (c) fill: the same interiors with every non-Sommerfeld halo poisoned
    Qp = Qo.copy()
    nlev = {lev: [w.n0[a] * 3 ** lev for a in range(3)] for lev in np.unique(m.ids[:, 0])}
    for p, (lev, i, j, k) in enumerate(m.ids):
        for a, idx in enumerate((i, j, k)):
            for side, sl in ((0, slice(0, 3)), (1, slice(12, 15))):
                phys = (idx == 0 and side == 0) or (idx == nlev[lev][a] - 1 and side == 1)
                if phys and w.bc == ccz4.BC_SOMMERFELD:
                    continue
                cut = [slice(3, 12)] * 3
                cut[2 - a] = sl
                Qp[(p,) + tuple(cut)] = np.nan
    Qd = to_gpu(Qp)
    del Qp
    ctx.fill_halos(Qd)
    g = to_host(Qd, sel)
    e = parity_error(g, Qo[sel], SLABS)
    assert e.max() <= 1e-13, ("fill", e.argmax(), e.max())
    del Qd
    # (b) init of the sampled leaves
    Qi = ctx.new_state(0.0)
    ctx.init_patches(Qi, w.scenario, w.scen)
    e = parity_error(to_host(Qi, sel), Qo[sel], INTERIOR)
    assert e.max() <= 1e-13, ("init", e.argmax(), e.max())


def test_full_size_step_graph_sampled():
    """The single puncture on its full 16^3-leaf mesh, one RK4 step in the launch configuration
    of the benchmark (autotuned fused stage kernel and block order, the step's halo flags, the
    captured step graph), against the oracle's RK4 step on the whole mesh, compared on sampled
    leaves: the interior, and the Sommerfeld ghost slabs of boundary leaves."""
    w = scenarios.config(2)
    ctx, m = make_pair(w.n0, w.origin, w.extent, w.bc, w.params(), w.refined)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    m.fill_halos(Qo)
    m.set_background(Qo)
    sel = _sample_patches(m.ids)
    Q0 = Qo[sel].copy()
    Qd = to_gpu(Qo)
    ctx.set_background(Qd)
    ctx.autotune(Qd, reps=1)
    ctx.fill_halos(Qd)
    dt = w.dt()
    Qo = m.rk4_step(oparams(w.params()), Qo, dt)
    ref = Qo[sel].copy()
    del Qo
    bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    g = ctx.step_graph(Qd, bufs, dt)
    g.launch()
    torch.cuda.synchronize()
    g.close()
    del bufs
    got = to_host(Qd, sel)
    del Qd
    e = parity_error(got, ref, INTERIOR)
    assert e.max() <= 1e-11, ("interior", e.argmax(), e.max())
    bm = boundary_ghost_mask(m, w.n0)[sel]
    eg = parity_error(np.where(bm[..., None], got, 0.0), np.where(bm[..., None], ref, 0.0), SLABS)
    assert eg.max() <= 1e-11, ("ghosts", eg.argmax(), eg.max())
    assert bm.any()
    # the step moved the state: the comparison is not one of unchanged data
    assert np.abs(ref[:, 3:12, 3:12, 3:12] - Q0[:, 3:12, 3:12, 3:12]).max() > 1e-10


def _subbox_oracle(w, ijk, margin=2):
    """An oracle mesh of the level-0 leaves within `margin` leaves of leaf ijk (clipped to the
    domain), with the workload's spacing, boundary condition and initial data: one RK4 step
    moves information 12 cells (four stages of reach 3), less than the 18 cells of two leaves,
    so the step's result on leaf ijk does not see the sub-box's own faces inside the domain."""
    L = w.extent[0] / w.n0[0]
    lo = [max(0, c - margin) for c in ijk]
    n = [min(w.n0[a] - 1, ijk[a] + margin) - lo[a] + 1 for a in range(3)]
    m = orc.Mesh(tuple(n), tuple(w.origin[a] + lo[a] * L for a in range(3)), tuple(n[a] * L for a in range(3)), w.bc)
    Q = m.zeros()
    m.init(Q, w.scenario, w.scen)
    return m, lo, Q


def nonzero_perturbed_runs(fn, Q, trials=2, seed=1234):
    """perturbed_runs with the zeros of Q left alone (one unit in the last place of a zero is a
    subnormal number, which slows the oracle's arithmetic many times over on a large box)."""
    return [fn(np.where(Q == 0.0, Q, ulp_perturbed(Q, seed + t))) for t in range(trials)]


def _full_size_config4_step(samples, precision, advection=0):
    """One captured RK4 step of the 24^3-leaf puncture in the benchmark's launch configuration for
    the precision; returns the GPU's sampled leaves after the step, per sample the oracle sub-box
    (mesh, initial state, index of the sampled leaf), and each slot's largest magnitude over the
    interiors of the whole mesh after the step."""
    w = scenarios.config(4)
    prm = ccz4.params(**{**w.prm, "advection": advection})
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, prm, w.refined)
    assert ctx.n_patches == 13824
    index = {tuple(r[1:]): p for p, r in enumerate(ctx.ids)}
    Qd = ctx.new_state(0.0)
    ctx.init_patches(Qd, w.scenario, w.scen)
    subs = []
    for ijk in samples:
        m, lo, Q = _subbox_oracle(w, ijk)
        full = [index[(r[1] + lo[0], r[2] + lo[1], r[3] + lo[2])] for r in m.ids]
        np.testing.assert_array_equal(ctx.geom[full], m.geom)  # the same leaves, bit for bit
        Qd[torch.tensor(full, device="cuda")] = to_gpu(Q)
        here = [p for p, r in enumerate(m.ids) if (r[1] + lo[0], r[2] + lo[1], r[3] + lo[2]) == ijk][0]
        subs.append((m, Q, here, index[ijk]))
    ctx.set_background(Qd)  # the boundary background of the uploaded leaves, as on the oracle side
    ctx.fill_halos(Qd)
    ctx.autotune(Qd, precision, reps=1)
    ctx.fill_halos(Qd)
    bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    g = ctx.step_graph(Qd, bufs, w.dt(), precision)
    g.launch()
    torch.cuda.synchronize()
    g.close()
    del bufs
    got = to_host(Qd, [s[3] for s in subs])
    mesh_scale = np.array([float(Qd[:, v, 3:12, 3:12, 3:12].abs().max()) for v in range(ccz4.NV)])
    del Qd
    torch.cuda.empty_cache()
    return w, prm, got, [s[:3] for s in subs], mesh_scale


def _domain_ghost_mask(w, ijk):
    """The sampled leaf's ghost slabs on the domain's faces."""
    bm = np.zeros((1, 15, 15, 15), bool)
    for a, c in enumerate(ijk):
        for side, cut_a in ((c == 0, slice(0, 3)), (c == w.n0[a] - 1, slice(12, 15))):
            if side:
                cut = [slice(3, 12)] * 3
                cut[2 - a] = cut_a
                bm[(0,) + tuple(cut)] = True
    return bm


def _check_full_size_fp64(samples, advection=0):
    """The FP64 step of _full_size_config4_step against the oracle on the sampled leaves: interior
    and Sommerfeld ghost slabs at 1e-11 (cancellation residuals: four times the oracle's one-ulp
    sensitivity)."""
    w, prm, got, subs, _ = _full_size_config4_step(samples, ccz4.PREC_FP64, advection)
    pr = oparams(prm)
    dt = w.dt()
    for n, (m, Q, here) in enumerate(subs):
        m.set_background(Q)
        m.fill_halos(Q)

        def run(Q0, m=m):
            return m.rk4_step(pr, Q0, dt)
        Q0 = Q.copy()
        ref = run(Q0.copy())
        r1, g1 = ref[here:here + 1], got[n:n + 1]
        runs = None
        e = parity_error(g1, r1, INTERIOR)
        if e.max() > 1e-11:  # a cancellation residual: the oracle's own one-ulp sensitivity decides
            runs = nonzero_perturbed_runs(run, Q0)
            e = parity_error(g1, r1, INTERIOR, sens=sensitivity(r1, [r[here:here + 1] for r in runs]), tol=1e-11)
        assert e.max() <= 1e-11, (samples[n], "interior", e.argmax(), e.max())
        bm = _domain_ghost_mask(w, samples[n])
        if bm.any():
            gh = lambda a: np.where(bm[..., None], a, 0.0)  # noqa: E731
            eg = parity_error(gh(g1), gh(r1), SLABS)
            if eg.max() > 1e-11:
                runs = runs or nonzero_perturbed_runs(run, Q0)
                eg = parity_error(gh(g1), gh(r1), SLABS, tol=1e-11,
                                  sens=sensitivity(gh(r1), [gh(r[here:here + 1]) for r in runs], SLABS))
            assert eg.max() <= 1e-11, (samples[n], "ghosts", eg.argmax(), eg.max())
        # the step moved the state
        assert np.abs(r1[:, 3:12, 3:12, 3:12] - Q0[here:here + 1, 3:12, 3:12, 3:12]).max() > 1e-10


def test_full_size_step_graph_config4_sampled():
    """The single puncture on its full 24^3-leaf mesh (13,824 leaves, 23.5 GB per state), one RK4
    step in the launch configuration of the benchmark (autotuned stage kernel, block and leaf
    order, the step's halo flags, the captured step graph), against the oracle on sampled leaves.
    The oracle cannot step the whole mesh in a test, so each sampled leaf is stepped on an oracle
    sub-box of the leaves around it; the sub-box's initial data (bit-identical geometry) are
    uploaded into the GPU state, so that both sides start from the same values wherever the
    sampled leaf's step can look.  Samples: the two domain corners, the leaves at the puncture,
    a boundary face and edge leaf, an interior leaf."""
    _check_full_size_fp64([(0, 0, 0), (23, 23, 23), (11, 11, 11), (12, 12, 12), (0, 12, 23), (5, 17, 9)])


def test_full_size_lopsided_step_graph_config4_sampled():
    """The same full-size check with lopsided advection (the upwind pairing of App. D's stencils,
    the benchmark's lopsided leg): a domain corner, the leaf at the puncture, an interior leaf."""
    _check_full_size_fp64([(0, 0, 0), (12, 12, 12), (5, 17, 9)], advection=1)


# Mixed precision at the benchmark's resolution (dx = 1/12): the cells next to the puncture carry
# terms in the right-hand sides of K, D and Theta that exceed those slots' sizes on the mesh far
# more than on the coarse test meshes, and the FP32 rounding of those terms is what the mixed state
# carries.  After one step there it reaches 1.9e-5 of Theta's size on the mesh (a cancellation
# residual of the Ricci scalar and the K terms) and 3.4e-6 for D; the bound stated for the leaves
# at the puncture on this mesh is 1e-4.  Away from them the bound of the test meshes holds.
MIXED_BOUND_PUNCTURE = 1e-4


def test_full_size_mixed_precision_step_graph_config4_sampled():
    """Mixed precision (FP32 algebra) at the benchmark's size and in its launch configuration for
    that precision: one captured RK4 step of the 24^3-leaf puncture against the FP64 oracle on
    sampled leaves (sub-boxes as in the FP64 test), on the interior and the Sommerfeld ghost slabs.
    The measure is relative to each slot's size on the mesh, as in the small-mesh test, where the
    compared cells are the whole mesh: the FP32 rounding of the algebra scales with the terms that
    feed a slot, not with the slot's value on one far-field leaf (there a slot such as D may be
    orders of magnitude below its size near the puncture).  Each slot's size is its largest
    interior magnitude over the 13,824 leaves after the step, with the floor of the parity
    measure.  A domain corner and an interior leaf are held to the test meshes' bound, the leaf at
    the puncture to the bound stated for it at this resolution."""
    samples = [(0, 0, 0), (12, 12, 12), (5, 17, 9)]
    bounds = [MIXED_BOUND, MIXED_BOUND_PUNCTURE, MIXED_BOUND]
    w, prm, got, subs, mesh_scale = _full_size_config4_step(samples, ccz4.PREC_MIXED)
    top = mesh_scale.max()
    scale = np.where(mesh_scale > FLOOR * top, mesh_scale, top)
    pr = oparams(prm)
    worst = 0.0
    for n, (m, Q, here) in enumerate(subs):
        m.set_background(Q)
        m.fill_halos(Q)
        ref = m.rk4_step(pr, Q.copy(), w.dt())
        r1, g1 = ref[here:here + 1], got[n:n + 1]
        e = np.abs(g1[:, INTERIOR] - r1[:, INTERIOR]).reshape(-1, ccz4.NV).max(0) / scale
        print(f"mixed vs oracle, leaf {samples[n]} of the 24^3-leaf mesh: max {e.max():.3e} at slot {e.argmax()}")
        assert e.max() <= bounds[n], (samples[n], "interior", e.argmax(), e.max())
        worst = max(worst, e.max())
        bm = _domain_ghost_mask(w, samples[n])
        if bm.any():
            eg = np.abs(g1[0][bm[0]] - r1[0][bm[0]]).max(0) / scale
            assert eg.max() <= bounds[n], (samples[n], "ghosts", eg.argmax(), eg.max())
    assert worst > 1e-12  # the FP32 algebra shows: the bound is not met trivially


# ------------------------------------------------------------------ fused stage

def _fused_vs_oracle(w, n0, refined=(), steps=2, perturb=False, kernel=ccz4.KERNEL_LDS, push=True):
    ctx, m = make_pair(n0, w.origin, w.extent, w.bc, w.params(), refined, kernel=kernel)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    if perturb:
        for p in range(m.np):
            Qo[p, 3:12, 3:12, 3:12] += 1e-3 * smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), 50)[3:12, 3:12, 3:12]
    Qd = to_gpu(Qo)
    ctx.set_background(to_gpu(Qo))
    m.set_background(Qo)
    ctx.fill_halos(Qd)
    bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    pr = oparams(w.params())
    dt = w.dt()

    def run(Q):
        for _ in range(steps):
            Q = m.rk4_step(pr, Q, dt)
        return Q
    for _ in range(steps):
        ctx.rk4_step_fused(Qd, dt, bufs, push=push)
    Q0 = Qo
    Qo = run(Q0.copy())
    # the oracle's own sensitivity to one-ulp changes of the initial state (gpu_helpers.KAPPA)
    runs = perturbed_runs(run, Q0)
    g = to_host(Qd)
    eg = np.zeros(59)
    if w.bc == ccz4.BC_SOMMERFELD:
        bm = boundary_ghost_mask(m, n0)
        gh = lambda a: np.where(bm[..., None], a, 0.0)  # noqa: E731
        eg = parity_error(gh(g), gh(Qo), SLABS, sens=sensitivity(gh(Qo), [gh(r) for r in runs], SLABS), tol=1e-11)
    return parity_error(g, Qo, INTERIOR, sens=sensitivity(Qo, runs), tol=1e-11), eg, ctx, Qd


def boundary_ghost_mask(m, n0):
    """(n, 15, 15, 15) mask of the ghost slabs of faces on the domain boundary."""
    out = np.zeros((m.np, 15, 15, 15), bool)
    for p, (lev, i, j, k) in enumerate(m.ids):
        for a, idx in enumerate((i, j, k)):
            na = n0[a] * 3 ** lev
            for side, sl in ((0, slice(0, 3)), (1, slice(12, 15))):
                if (side == 0 and idx == 0) or (side == 1 and idx == na - 1):
                    cut = [slice(3, 12)] * 3
                    cut[2 - a] = sl
                    out[(p,) + tuple(cut)] = True
    return out


@pytest.mark.parametrize("push", [True, False])
@pytest.mark.parametrize("kernel", KERNELS)
def test_fused_stage_config1_matches_oracle(kernel, push):
    w = scenarios.config(1)
    e, _, _, _ = _fused_vs_oracle(w, w.n0, steps=10, kernel=kernel, push=push)
    assert e.max() <= 1e-11, (e.argmax(), e.max())


@pytest.mark.parametrize("push", [True, False])
@pytest.mark.parametrize("kernel", KERNELS)
def test_fused_stage_puncture_sommerfeld_matches_oracle(kernel, push):
    w = scenarios.config(2)
    e, eg, _, _ = _fused_vs_oracle(w, (2, 2, 2), steps=2, perturb=True, kernel=kernel, push=push)
    assert e.max() <= 1e-11, (e.argmax(), e.max())
    assert eg.max() <= 1e-11, (eg.argmax(), eg.max())


@pytest.mark.parametrize("kernel", KERNELS)
def test_fused_stage_amr_matches_unfused_gpu_path(kernel):
    """Fused and unfused GPU steps on a mesh with coarse-fine faces agree (the oracle's own AMR
    step is checked by the sampled tests); differences come from summation order only."""
    w = scenarios.config(2)
    refined = [(0, 1, 1, 1)]
    ctx = ccz4.Context((3, 3, 3), (-9.0,) * 3, (18.0,) * 3, w.bc, w.params(), refined)
    ctx.set_kernel(ccz4.PREC_FP64, kernel)
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    ctx.fill_halos(Q)
    Q2 = Q.clone()
    b1 = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    b2 = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    dt = 0.1 * 18.0 / 81 / 3
    for _ in range(2):
        ctx.rk4_step_fused(Q, dt, b1)
        ctx.rk4_step(Q2, dt, b2)
    e = parity_error(to_host(Q), to_host(Q2), INTERIOR)
    assert e.max() <= 1e-13, (e.argmax(), e.max())
    # the fused step with halo push leaves Q's halos filled; the unfused one leaves them from
    # before its last stage: after a fill of the latter both agree on the halo slabs as well
    Qf = Q.clone()
    ctx.fill_halos(Q2)
    ctx.fill_halos(Qf)
    assert torch.equal(Qf, Q)
    e = parity_error(to_host(Q), to_host(Q2), INTERIOR | SLABS)
    assert e.max() <= 1e-13, (e.argmax(), e.max())


def test_fused_stage_rejects_aliasing():
    ctx = ccz4.Context((1, 1, 1), (0, 0, 0), (1.0, 1.0, 1.0), ccz4.BC_PERIODIC, ccz4.params())
    a, b, c = ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0)
    for args in ((0, 0.1, a, a, b, a), (1, 0.1, a, b, c, b), (0, 0.1, a, b, a, c), (0, -1.0, a, b, c, a)):
        with pytest.raises(ccz4.CCZ4Error):
            ctx.rhs_rk4_stage(*args)


@pytest.mark.parametrize("kernel", KERNELS)
def test_fused_steps_static_amr_first_order_app_e_match_oracle(kernel):
    """First-order formulation with the App. E coarse-fine operators on a static two-level mesh
    with Sommerfeld faces: fused RK4 steps against the oracle's steps, interior and ghost slabs.
    The refined cube [-9, 0]^3 has the puncture at its corner, so no cell centre falls on it."""
    w = scenarios.config(2)
    e, eg, _, _ = _fused_vs_oracle(w, (2, 2, 2), refined=[(0, 0, 0, 0)], steps=2, perturb=True, kernel=kernel)
    assert e.max() <= 1e-11, (e.argmax(), e.max())
    assert eg.max() <= 1e-11, (eg.argmax(), eg.max())


# Mixed precision (FP32 nonlinear algebra; FP64 state, stencil differences, metric inverse and
# determinant, 1/phi factors and RK accumulation) against the FP64 oracle: after two RK4 steps
# of the perturbed puncture, the per-slot error of the parity measure stays below MIXED_BOUND.
# The bound is FP32 rounding (6e-8) of the algebra's terms, each of which can be larger than the
# slot it feeds (the Ricci sum against alpha R / 2 of Theta), times the two steps' accumulation.
MIXED_BOUND = 1e-6


@pytest.mark.parametrize("refined", [(), ((0, 0, 0, 0),)], ids=["uniform", "two_levels"])
@pytest.mark.parametrize("kernel", KERNELS)
def test_mixed_precision_steps_against_oracle(kernel, refined):
    w = scenarios.config(2)
    ctx, m = make_pair((2, 2, 2), w.origin, w.extent, w.bc, w.params(), list(refined))
    ctx.set_kernel(ccz4.PREC_MIXED, kernel)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    for p in range(m.np):
        Qo[p, 3:12, 3:12, 3:12] += 1e-3 * smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), 50)[3:12, 3:12, 3:12]
    Qd = to_gpu(Qo)
    ctx.set_background(to_gpu(Qo))
    m.set_background(Qo)
    ctx.fill_halos(Qd)
    bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    pr = oparams(w.params())
    dt = w.dt()
    for _ in range(2):
        ctx.rk4_step_fused(Qd, dt, bufs, ccz4.PREC_MIXED)
        Qo = m.rk4_step(pr, Qo, dt)
    g = to_host(Qd)
    e = parity_error(g, Qo, INTERIOR)
    print(f"mixed vs oracle ({kernel}, {len(refined)} refined): max {e.max():.3e} at slot {e.argmax()}")
    assert e.max() <= MIXED_BOUND, (e.argmax(), e.max())
    bm = boundary_ghost_mask(m, (2, 2, 2))
    eg = parity_error(np.where(bm[..., None], g, 0.0), np.where(bm[..., None], Qo, 0.0), SLABS)
    assert eg.max() <= MIXED_BOUND, (eg.argmax(), eg.max())
    # the mixed path differs from the FP64 one: the bound is not met trivially
    assert e.max() > 1e-12


def test_kernels_agree_on_a_static_amr_mesh():
    """Both right-hand-side kernels on every leaf of a two-level mesh with Sommerfeld faces,
    random smooth state: they agree with each other to rounding, and the LDS kernel with the
    oracle, for both the plain RHS and one fused stage."""
    w = scenarios.config(2)
    refined = [(0, 1, 1, 1), (0, 2, 1, 1)]
    ctx, m = make_pair((4, 3, 3), (-9.0, -6.75, -6.75), (18.0, 13.5, 13.5), w.bc, w.params(), refined)
    Qo = random_state(m, 61)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    ctx.set_background(Qd)
    k_ph, k_lds = ctx.new_state(0.0), ctx.new_state(0.0)
    ctx.set_kernel(ccz4.PREC_FP64, ccz4.KERNEL_PHASED)
    ctx.rhs(Qd, k_ph)
    ctx.set_kernel(ccz4.PREC_FP64, ccz4.KERNEL_LDS)
    ctx.rhs(Qd, k_lds)
    e = parity_error(to_host(k_lds), to_host(k_ph), INTERIOR)
    assert e.max() <= 1e-13, (e.argmax(), e.max())
    e = parity_error(to_host(k_lds), m.rhs(oparams(w.params()), Qo), INTERIOR)
    assert e.max() <= TOL, (e.argmax(), e.max())
    outs = []
    for kern in KERNELS:
        ctx.set_kernel(ccz4.PREC_FP64, kern)
        acc, Qx = ctx.new_state(0.0), ctx.new_state(0.0)
        ctx.rhs_rk4_stage(1, 0.01, Qd, Qd.clone(), acc, Qx)
        outs.append((acc, to_host(Qx)))
    e = parity_error(outs[1][1], outs[0][1], INTERIOR)
    assert e.max() <= 1e-13, (e.argmax(), e.max())
    e = acc_slot_error(outs[1][0], outs[0][0])
    assert e.max() <= 1e-13, (e.argmax(), e.max())


def test_kernel_selection_rejects_bad_arguments():
    ctx = ccz4.Context((1, 1, 1), (0, 0, 0), (1.0, 1.0, 1.0), ccz4.BC_PERIODIC, ccz4.params())
    for args in ((2, 0), (0, ccz4.KERNEL_CONFIGS), (-1, 1), (0, -1)):
        with pytest.raises(ccz4.CCZ4Error):
            ctx.set_kernel(*args)
    assert ctx.get_kernel(ccz4.PREC_FP64) == ccz4.KERNEL_LDS


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("periodic", [True, False])
def test_stage_push_writes_exactly_the_same_level_halos(kernel, periodic):
    """A fused stage with CCZ4_STAGE_FILL_SAME_LEVEL leaves Qnext bit-identical to the same stage
    without it followed by the same-level fill (s = 1 and the projected s = 3), on a mesh with
    coarse-fine faces (left for the level fill) and periodic self-neighbours or Sommerfeld faces."""
    if periodic:
        w = scenarios.config(1)
        ctx = ccz4.Context((1, 2, 3), (-0.5, -0.5, -0.5), (1.0 / 3, 2.0 / 3, 1.0), ccz4.BC_PERIODIC, w.params())
        Q = ctx.new_state(0.0)
        ctx.init_patches(Q, w.scenario, w.scen)
    else:
        w = scenarios.config(2)
        ctx = ccz4.Context((3, 3, 2), (-9.0, -9.0, -6.0), (18.0, 18.0, 12.0), w.bc, w.params(), [(0, 1, 1, 0)])
        Q = ctx.new_state(0.0)
        ctx.init_patches(Q, w.scenario, w.scen)
    counts = ctx.plan_counts()
    assert counts["same_level"] > 0
    if not periodic:
        assert counts["restrict"] > 0 and counts["prolong"] > 0 and counts["sommerfeld"] > 0
    ctx.set_kernel(ccz4.PREC_FP64, kernel)
    ctx.fill_halos(Q)
    acc0 = valid_accumulator(ctx, Q)
    for s in (1, 3):
        acc = acc0.clone()
        a_push, a_ref = ctx.new_state(0.0), ctx.new_state(0.0)
        acc2 = acc.clone()
        ctx.rhs_rk4_stage(s, 0.01, Q, Q, acc, a_push, ccz4.PREC_FP64, ccz4.STAGE_FILL_SAME_LEVEL)
        ctx.rhs_rk4_stage(s, 0.01, Q, Q, acc2, a_ref, ccz4.PREC_FP64, 0)
        ctx.fill_halos_kinds(a_ref, ccz4.FILL_SAME_LEVEL)
        assert bool(torch.isfinite(a_ref).all()), s
        bad = (a_push != a_ref).nonzero()
        assert bad.shape[0] == 0, (s, bad.shape[0], bad[:5].tolist())
        assert torch.equal(acc, acc2), s
    with pytest.raises(ccz4.CCZ4Error):
        ctx.rhs_rk4_stage(1, 0.01, Q, Q, acc, a_push, ccz4.PREC_FP64, 8)
    with pytest.raises(ccz4.CCZ4Error):
        ctx.fill_halos_kinds(Q, 8)


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("push", [False, True])
def test_stage_gather_reads_same_level_halos_from_the_neighbours(periodic, push):
    """With CCZ4_STAGE_GATHER_SAME_LEVEL the fused stage reads every same-level y and z face halo
    of Qs from the neighbour's interior: with those halos of Qs overwritten by NaN it gives Qnext
    and the accumulator bit-identical to the stage on the filled state (s = 0, 1 and the projected
    s = 3), on a mesh of periodic self-neighbours and on one with coarse-fine and Sommerfeld
    faces (whose own halos it still reads), with and without the halo push."""
    if periodic:
        w = scenarios.config(1)
        ctx = ccz4.Context((1, 2, 3), (-0.5, -0.5, -0.5), (1.0 / 3, 2.0 / 3, 1.0), ccz4.BC_PERIODIC, w.params())
    else:
        w = scenarios.config(2)
        ctx = ccz4.Context((3, 3, 2), (-9.0, -9.0, -6.0), (18.0, 18.0, 12.0), w.bc, w.params(), [(0, 1, 1, 0)])
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    ctx.fill_halos(Q)
    ctx.set_kernel(ccz4.PREC_FP64, ccz4.KERNEL_LDS)
    mask = same_level_halo_mask(ctx, Q, axes=(1, 2))
    assert int(mask.sum()) > 0
    G = Q.clone()
    G[mask] = float("nan")
    acc0 = valid_accumulator(ctx, Q)
    fl = ccz4.STAGE_FILL_SAME_LEVEL if push else 0
    for s in (0, 1, 3):
        acc_r, acc_g = acc0.clone(), acc0.clone()
        out_r, out_g = ctx.new_state(0.0), ctx.new_state(0.0)
        ctx.rhs_rk4_stage(s, 0.01, Q, Q, acc_r, out_r, ccz4.PREC_FP64, fl)
        ctx.rhs_rk4_stage(s, 0.01, G, Q, acc_g, out_g, ccz4.PREC_FP64, fl | ccz4.STAGE_GATHER_SAME_LEVEL)
        assert bool(torch.isfinite(out_g).all()), s
        assert torch.equal(out_g, out_r), (s, int((out_g != out_r).sum()))
        assert torch.equal(acc_g, acc_r), s
    # the phased kernel reads its own halos: gathering is refused
    ctx.set_kernel(ccz4.PREC_FP64, ccz4.KERNEL_PHASED)
    with pytest.raises(ccz4.CCZ4Error):
        ctx.rhs_rk4_stage(1, 0.01, Q, Q, acc0, out_r, ccz4.PREC_FP64, ccz4.STAGE_GATHER_SAME_LEVEL)
    with pytest.raises(ccz4.CCZ4Error):
        ctx.rhs_rk4_stage(1, 0.01, Q, Q, acc0, out_r, ccz4.PREC_FP64, 8)


@pytest.mark.parametrize("kernel", KERNELS)
def test_stage_push_x_writes_exactly_the_x_face_halos(kernel):
    """CCZ4_STAGE_FILL_SAME_LEVEL_X writes the same-level x-face halos of Qnext exactly as the full
    push does, and no y or z face halo."""
    w = scenarios.config(2)
    ctx = ccz4.Context((3, 3, 2), (-9.0, -9.0, -6.0), (18.0, 18.0, 12.0), w.bc, w.params(), [(0, 1, 1, 0)])
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    ctx.fill_halos(Q)
    ctx.set_kernel(ccz4.PREC_FP64, kernel)
    acc0 = valid_accumulator(ctx, Q)
    full, xonly, none = ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0)
    for out, fl in ((full, ccz4.STAGE_FILL_SAME_LEVEL), (xonly, ccz4.STAGE_FILL_SAME_LEVEL_X), (none, 0)):
        ctx.rhs_rk4_stage(1, 0.01, Q, Q, acc0.clone(), out, ccz4.PREC_FP64, fl)
    mx = same_level_halo_mask(ctx, Q, axes=(0,))
    assert int(mx.sum()) > 0
    assert torch.equal(xonly[mx], full[mx])
    assert torch.equal(xonly[~mx], none[~mx])


def test_step_stage_flags():
    """The flags of a step's stages (and second-order reconstructions): the LDS kernel gathers the
    y and z halos at every stage and copies the x-face halos at s = 0..2 and all of them at s = 3;
    the phased kernel copies every face after every stage."""
    G, F, X = ccz4.STAGE_GATHER_SAME_LEVEL, ccz4.STAGE_FILL_SAME_LEVEL, ccz4.STAGE_FILL_SAME_LEVEL_X
    for form, want in ((ccz4.FORMULATION_FO, [G | X, G | X, G | X, G | F]),
                       (ccz4.FORMULATION_SO, [G | X, G | X, G | X, G | F])):
        ctx = ccz4.Context((2, 1, 1), (0.0, 0.0, 0.0), (2.0, 1.0, 1.0), ccz4.BC_PERIODIC,
                           ccz4.params(formulation=form))
        for prec in (ccz4.PREC_FP64, ccz4.PREC_MIXED):
            ctx.set_kernel(prec, ccz4.KERNEL_LDS)
            assert [ctx.step_stage_flags(s, prec) for s in range(4)] == want
            ctx.set_kernel(prec, ccz4.KERNEL_PHASED)
            assert [ctx.step_stage_flags(s, prec) for s in range(4)] == [F] * 4
        for bad in ((-1, 0), (4, 0), (0, 2)):
            with pytest.raises(ccz4.CCZ4Error):
                ctx.step_stage_flags(*bad)


def test_autotune_block_and_leaf_order():
    """The autotuner times the sixteen launch configurations (kernel, block order, leaf order) and
    keeps the fastest; neither order changes the arithmetic (bit-identical stages for one kernel),
    and the two kernels agree to rounding."""
    w = scenarios.config(2)
    ctx = ccz4.Context((3, 3, 2), (-9.0, -9.0, -6.0), (18.0, 18.0, 12.0), w.bc, w.params(), [(0, 1, 1, 0)])
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    ctx.fill_halos(Q)
    ms = ctx.autotune(Q, ccz4.PREC_FP64, reps=2)
    assert len(ms) == ccz4.KERNEL_CONFIGS and all(t > 0 for t in ms)
    assert ctx.get_kernel(ccz4.PREC_FP64) == int(np.argmin(ms))
    outs = {}
    for k in range(ccz4.KERNEL_CONFIGS):
        ctx.set_kernel(ccz4.PREC_FP64, k)
        acc, Qx = Q.clone(), ctx.new_state(0.0)
        ctx.rhs_rk4_stage(1, 0.01, Q, Q, acc, Qx, ccz4.PREC_FP64, ccz4.STAGE_FILL_SAME_LEVEL)
        outs[k] = (acc, Qx)
    for k in range(2, ccz4.KERNEL_CONFIGS):
        assert torch.equal(outs[k][0], outs[k % 2][0]) and torch.equal(outs[k][1], outs[k % 2][1]), k
    e = parity_error(to_host(outs[0][1]), to_host(outs[1][1]), INTERIOR | SLABS)
    assert e.max() <= 1e-13, e.max()
    # the standalone right-hand side in every configuration
    k0 = ctx.new_state(0.0)
    ctx.set_kernel(ccz4.PREC_FP64, ccz4.KERNEL_LDS)
    ctx.rhs(Q, k0)
    for k in (ccz4.KERNEL_LDS | ccz4.KERNEL_ORDER_MORTON, ccz4.KERNEL_LDS | ccz4.KERNEL_ORDER_Z_PENCILS,
              ccz4.KERNEL_LDS | ccz4.KERNEL_LINEAR_ORDER | ccz4.KERNEL_ORDER_BRICKS):
        ctx.set_kernel(ccz4.PREC_FP64, k)
        k1 = ctx.new_state(0.0)
        ctx.rhs(Q, k1)
        assert torch.equal(k1, k0), k
    with pytest.raises(ccz4.CCZ4Error):
        ctx.set_kernel(ccz4.PREC_FP64, ccz4.KERNEL_CONFIGS)


@pytest.mark.parametrize("kernel", KERNELS)
def test_step_graph_replays_match_eager_steps(kernel):
    """The captured RK4 step, replayed several times with eager work and synchronisation in
    between, equals the eager fused step bit for bit after every replay."""
    w = scenarios.config(2)
    ctx = ccz4.Context((3, 3, 2), (-9.0, -9.0, -6.0), (18.0, 18.0, 12.0), w.bc, w.params(), [(0, 1, 1, 0)])
    ctx.set_kernel(ccz4.PREC_FP64, kernel)
    Qg = ctx.new_state(0.0)
    ctx.init_patches(Qg, w.scenario, w.scen)
    ctx.fill_halos(Qg)
    Qe = Qg.clone()
    dt = 0.1 * 18.0 / 27 / 9
    bg = tuple(ctx.new_state(0.0) for _ in range(3))
    be = tuple(ctx.new_state(0.0) for _ in range(3))
    graph = ctx.step_graph(Qg, bg, dt)
    for rep in range(3):
        graph.launch()
        torch.cuda.synchronize()
        ctx.rk4_step_fused(Qe, dt, be)
        torch.cuda.synchronize()
        assert torch.equal(Qg, Qe), rep
        norms, _ = ctx.constraints(Qe)  # unrelated eager work between replays
    graph.close()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_regrid_plan_and_transfer_match_oracle(seed):
    """Regrid of a Sommerfeld mesh with two levels under random tags: the library's plan equals
    the oracle's (integer work: exactly), and the transferred state equals the oracle's bit for
    bit on every new leaf (whole box for kept leaves, interior for the others)."""
    w = scenarios.config(2)
    refined = [(0, 1, 1, 1), (0, 2, 2, 1), (1, 4, 4, 4)]
    n0, org, ext = (4, 4, 3), (-9.0, -9.0, -6.75), (18.0, 18.0, 13.5)
    ctx, m = make_pair(n0, org, ext, w.bc, w.params(), refined)
    rng = np.random.default_rng(80 + seed)
    tags = rng.choice(np.array([-1, 0, 0, 1], np.int8), m.np)
    if seed == 0:  # one whole family asked to coarsen
        tags[m.ids[:, 0] == 2] = -1
    plan_d = ccz4.ccz4_regrid_plan(ctx.h, tags, 3)
    plan_o = m.regrid_plan(tags, 3)
    assert {tuple(r) for r in plan_d.tolist()} == {tuple(r) for r in plan_o.tolist()}
    new_refined = [tuple(int(v) for v in r) for r in plan_o]
    ctx2, m2 = make_pair(n0, org, ext, w.bc, w.params(), new_refined)
    Qo = random_state(m, 90 + seed)
    Qn_o = m2.zeros()
    m.regrid_transfer(Qo, m2, Qn_o)
    Qn_d = ctx2.new_state(0.0)
    ccz4.ccz4_regrid_transfer(ctx.h, to_gpu(Qo), ctx2.h, Qn_d)
    got = to_host(Qn_d)
    assert np.array_equal(got[:, 3:12, 3:12, 3:12], Qn_o[:, 3:12, 3:12, 3:12])
    kept = [p for p, idv in enumerate(m2.ids.tolist()) if idv in m.ids.tolist()]
    assert np.array_equal(got[kept], Qn_o[kept])

"""GPU parity of the lopsided advection stencils (App. D) against the oracle, for both pairings
(biased towards +x_k where beta^k > 0, and as printed) and both kernels: right-hand sides on
random states whose shift takes both signs, with the second-order formulation too, and whole
fused RK4 steps of the puncture.  Same 1e-12 normwise measure per slot as the central runs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as orc  # noqa: E402
from gpu_helpers import parity_error, to_gpu, to_host  # noqa: E402
from paper_2406_11626_amd import ccz4, scenarios  # noqa: E402
from seeded_inputs import box_centers, smooth_state  # noqa: E402

KERNELS = [ccz4.KERNEL_PHASED, ccz4.KERNEL_LDS]
MODES = [ccz4.ADVECTION_LOPSIDED_UPWIND, ccz4.ADVECTION_LOPSIDED_PRINTED]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ccz4.lib()


def oparams(prm):
    return orc.Params(**{f: getattr(prm, f) for f, _ in ccz4.Params._fields_})


def make_pair(n0, origin, extent, bc, prm, kernel):
    ctx = ccz4.Context(n0, origin, extent, bc, prm)
    for prec in (ccz4.PREC_FP64, ccz4.PREC_MIXED):
        ctx.set_kernel(prec, kernel)
    m = orc.Mesh(n0, origin, extent, bc)
    return ctx, m


@pytest.mark.parametrize("formulation", [0, 1])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("kernel", KERNELS)
def test_lopsided_rhs_parity_random_states(kernel, mode, formulation):
    prm = ccz4.params(advection=mode, formulation=formulation, kappa1=0.3, kappa3=0.5)
    ctx, m = make_pair((2, 2, 1), (-0.4, 0.1, 0.2), (1.6, 1.6, 0.8), ccz4.BC_PERIODIC, prm, kernel)
    Qo = m.zeros()
    for p in range(m.np):
        Qo[p] = smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), 60 + p)
    # the smooth shift changes sign inside the patches: both stencils of each pairing are taken
    assert (Qo[..., 7:10] > 0).any() and (Qo[..., 7:10] < 0).any()
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    kd = ctx.new_state(0.0)
    ctx.rhs(Qd, kd)
    ko = m.rhs(oparams(prm), Qo)
    e = parity_error(to_host(kd), ko)
    assert e.max() <= 1e-12, (e.argmax(), e.max())
    # and it differs from the central-advection right-hand side
    kc = m.rhs(oparams(ccz4.params(formulation=formulation, kappa1=0.3, kappa3=0.5)), Qo)
    assert np.abs(ko - kc)[:, 3:12, 3:12, 3:12, 11:25].max() > 1e-6


@pytest.mark.parametrize("kernel", KERNELS)
def test_lopsided_fused_steps_puncture_match_oracle(kernel):
    w = scenarios.config(2)
    prm = ccz4.params(**{**w.prm, "advection": ccz4.ADVECTION_LOPSIDED_UPWIND})
    ctx, m = make_pair((2, 2, 2), w.origin, w.extent, w.bc, prm, kernel)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    for p in range(m.np):  # a shift of both signs from the start
        Qo[p, 3:12, 3:12, 3:12] += 1e-3 * smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), 61)[3:12, 3:12, 3:12]
    m.set_background(Qo)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    ctx.set_background(to_gpu(Qo))
    bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    pr = oparams(prm)
    for _ in range(2):
        ctx.rk4_step_fused(Qd, w.dt(), bufs)
        Qo = m.rk4_step(pr, Qo, w.dt())
    e = parity_error(to_host(Qd), Qo)
    assert e.max() <= 1e-11, (e.argmax(), e.max())


def test_advection_parameter_is_checked():
    with pytest.raises(ccz4.CCZ4Error):
        ccz4.Context((1, 1, 1), (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), ccz4.BC_PERIODIC, ccz4.params(advection=3))

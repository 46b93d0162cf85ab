"""GPU parity of the higher-order coarse-fine operators (transfer = 1: injection restriction,
three-point quadratic prolongation) against the oracle: the halo fill on a two-level refined mesh
of both boundary kinds, and fused RK4 steps of the puncture on a static AMR mesh."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as orc  # noqa: E402
from gpu_helpers import SLABS, parity_error, to_gpu, to_host  # noqa: E402
from paper_2406_11626_amd import ccz4, scenarios  # noqa: E402
from seeded_inputs import box_centers, smooth_state  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ccz4.lib()


def pair(n0, origin, extent, bc, prm, refined):
    ctx = ccz4.Context(n0, origin, extent, bc, prm, refined)
    m = orc.Mesh(n0, origin, extent, bc, refined)
    m.set_transfer(prm.transfer)
    assert np.array_equal(ctx.ids, m.ids)
    return ctx, m


@pytest.mark.parametrize("bc", [ccz4.BC_PERIODIC, ccz4.BC_NEUMANN])
def test_fill_higher_order_matches_oracle(bc):
    refined = [(0, 1, 1, 1), (1, 4, 4, 4)]
    ctx, m = pair((3, 3, 3), (0, 0, 0), (3.0, 3.0, 3.0), bc, ccz4.params(transfer=1), refined)
    Qo = m.zeros()
    for p in range(m.np):
        Qo[p] = smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), 80)
    Qo[:, SLABS] = 0.0
    Qd = to_gpu(Qo)
    ctx.fill_halos(Qd)
    m.fill_halos(Qo)
    g = to_host(Qd)
    e = parity_error(g, Qo, SLABS)
    assert e.max() <= 1e-14, e.max()
    # and it is not the App. E result
    Q0 = Qo.copy()
    Q0[:, SLABS] = 0.0
    m0 = orc.Mesh((3, 3, 3), (0, 0, 0), (3.0, 3.0, 3.0), bc, refined)
    m0.fill_halos(Q0)
    assert np.abs(np.where(SLABS[..., None], Q0 - g, 0.0)).max() > 1e-8


def test_fused_steps_static_amr_higher_order_match_oracle():
    w = scenarios.config(2)
    prm = ccz4.params(**{**w.prm, "transfer": ccz4.TRANSFER_HIGHER_ORDER})
    # the refined cube [-9, 0]^3 has the puncture at its corner: no cell centre of either level
    # falls on it
    refined = [(0, 0, 0, 0)]
    ctx, m = pair((2, 2, 2), w.origin, w.extent, w.bc, prm, refined)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    for p in range(m.np):
        Qo[p, 3:12, 3:12, 3:12] += 1e-3 * smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), 81)[3:12, 3:12, 3:12]
    m.set_background(Qo)
    m.fill_halos(Qo)
    Qd = to_gpu(Qo)
    ctx.set_background(to_gpu(Qo))
    bufs = (ctx.new_state(0.0), ctx.new_state(0.0), ctx.new_state(0.0))
    pr = orc.Params(**{f: getattr(prm, f) for f, _ in ccz4.Params._fields_})
    for _ in range(2):
        ctx.rk4_step_fused(Qd, w.dt(), bufs)
        Qo = m.rk4_step(pr, Qo, w.dt())
    e = parity_error(to_host(Qd), Qo)
    assert e.max() <= 1e-11, (e.argmax(), e.max())

"""Work-buffer placement (Context.tune_step_buffers): the trial steps are ordinary fused steps, so
they advance the state exactly as the same number of fused steps on any other buffers does, and the
three buffers kept serve further steps with the same results.  The comparison steps run on work
buffers filled with NaN, which shows that no step reads what a work buffer held before it (a mesh
with a refined leaf and Sommerfeld boundaries, so the level fills and the ghost slabs take part)."""
import math

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2406_11626_amd import ccz4, scenarios  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ccz4.lib()


def test_tune_step_buffers_steps_like_fused_steps_on_any_buffers():
    w = scenarios.config(2)
    ctx = ccz4.Context((3, 3, 3), (-9.0,) * 3, (18.0,) * 3, w.bc, w.params(), [(0, 1, 1, 1)])
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    ctx.fill_halos(Q)
    R = Q.clone()
    dt = 0.1 * 18.0 / 81 / 3
    pool, steps = 4, 1
    keep, ms = ctx.tune_step_buffers(Q, dt, pool=pool, steps=steps)
    assert len(ms) == pool and all(t > 0 and math.isfinite(t) for t in ms)
    assert len({b.data_ptr() for b in keep} | {Q.data_ptr()}) == 4
    assert all(b.shape == Q.shape and b.dtype == torch.float64 for b in keep)
    nan = (ctx.new_state(math.nan), ctx.new_state(math.nan), ctx.new_state(math.nan))
    for _ in range(pool * steps):
        ctx.rk4_step_fused(R, dt, nan)
    torch.cuda.synchronize()
    assert torch.equal(Q, R)
    # two more steps: on the buffers kept, and on NaN-filled ones again
    nan = tuple(b.fill_(math.nan) for b in nan)
    for _ in range(2):
        ctx.rk4_step_fused(Q, dt, keep)
        ctx.rk4_step_fused(R, dt, nan)
    torch.cuda.synchronize()
    assert torch.equal(Q, R)
    assert bool(torch.isfinite(Q[:, :, 3:12, 3:12, 3:12]).all())

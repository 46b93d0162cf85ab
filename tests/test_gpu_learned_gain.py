"""What the learned refinement indicator gains over the plain criterion.

The plain criterion tags a leaf from its fields now; a regrid placed from those tags is late for
a feature that moves.  The network is trained, on the solver's own run, to predict the plain tag
one snapshot (60 steps) ahead from the leaf features now; combined with the plain criterion
(ccz4_tag_learned) it should place the refinement that the plain criterion will ask for next.

Training runs: gauge waves of amplitudes 0.07, 0.09, 0.11 and 0.13 (the paper's gauge-wave test,
moving along x at unit speed) on a periodic row of 9 patches with a static refined band at
patches 3-5, one period each.  Held-out runs: amplitudes 0.10 and 0.12 with the refined band at
patches 5-7, one period.  Score on the held-out runs: the fraction of leaves that the plain
criterion tags REFINE at snapshot k+1 and that the tags of snapshot k do not refine (miss rate), and the REFINE tags not asked for."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2406_11626_amd import ccz4, scenarios  # noqa: E402
from paper_2406_11626_amd.learned import LearnedIndicator, anticipation, snapshots  # noqa: E402

THETA_R, THETA_C = 0.003, 0.001


def gauge_run(amplitude, band, periods):
    n0, ext = (9, 1, 1), (1.0, 1.0 / 9, 1.0 / 9)
    ref = [(0, i, 0, 0) for i in band]
    ctx = ccz4.Context(n0, (-0.5, -1 / 18, -1 / 18), ext, ccz4.BC_PERIODIC, ccz4.params(**scenarios.GAUGE), ref)
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, ccz4.SCEN_GAUGE_WAVE, [amplitude, 2.0])
    ctx.fill_halos(Q)
    dt = 0.1 / 243  # CFL 0.1 on the finest level
    return ctx, snapshots(ctx, Q, dt, 2430 * periods, 60, THETA_R, THETA_C, 2)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ccz4.lib()


TRAIN_AMPLITUDES = (0.07, 0.09, 0.11, 0.13)
HELD_OUT = ((0.10, (5, 6, 7)), (0.12, (5, 6, 7)))
CONF = 0.6


def training_set():
    X, Y = [], []
    for a in TRAIN_AMPLITUDES:
        _, sn = gauge_run(a, (3, 4, 5), 1)
        X += [f for f, _ in sn[:-1]]
        Y += [t for _, t in sn[1:]]
    return torch.cat(X), torch.cat(Y)


def test_learned_indicator_anticipates_refinement():
    X, Y = training_set()
    counts = np.bincount(Y.cpu().numpy().astype(np.int64) + 1, minlength=3)
    assert counts.min() > 0, counts  # all three classes occur in the labels
    ind = LearnedIndicator(seed=0)
    ind.fit_normalisation(X)
    loss0 = ind.train(X, Y, 0)
    loss = ind.train(X, Y, 1500, lr=3e-3)
    assert loss < 0.25 * loss0, (loss0, loss)
    for amp, band in HELD_OUT:
        ctx_b, held = gauge_run(amp, band, 1)
        s = anticipation(ind, ctx_b, held, CONF)
        print("held-out", amp, "anticipation (miss rate, extra REFINE per snapshot):", s)
        miss_plain, extra_plain = s["plain"]
        miss_comb, extra_comb = s["combined"]
        assert miss_plain > 0.03  # the moving wave does make the plain criterion late
        assert miss_comb <= 0.5 * miss_plain, s
        # the gain is not bought by refining everything: at most two extra leaves per snapshot
        # on average, out of 87
        assert extra_comb <= extra_plain + 2.0, s

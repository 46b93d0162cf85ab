"""Dynamic AMR with the learned indicator inside the regrid loop (the plain refinement criterion
stays the fallback): with a network that is never confident (a zero output layer: probability
1/3 for every class, against a confidence threshold of 1) the combination is the plain
criterion, so the whole evolution (meshes and states) equals the plain one bit for bit; with a
network that is always confident every plain REFINE is kept and the network's own REFINE tags
are added, and the evolution stays finite."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2406_11626_amd import ccz4, dynamic, scenarios  # noqa: E402
from paper_2406_11626_amd.learned import LearnedIndicator  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ccz4.lib()


def workload():
    w = scenarios.config(5)
    return scenarios.Workload("binary puncture, 3^3 cubes on [-12,12]^3, two cubes refined", (3, 3, 3), w.origin,
                              w.extent, w.bc, w.prm, w.scenario, w.scen, 4, refined=[(0, 1, 1, 1), (0, 2, 1, 1)])


def start(w):
    ctx = ccz4.Context(w.n0, w.origin, w.extent, w.bc, w.params(), w.refined)
    Q = ctx.new_state(0.0)
    ctx.init_patches(Q, w.scenario, w.scen)
    ctx.fill_halos(Q)
    return ctx, Q


def thresholds(ctx, Q):
    ind = torch.empty((ctx.n_patches, 3), dtype=torch.float64, device="cuda")
    tags = torch.empty(ctx.n_patches, dtype=torch.int8, device="cuda")
    ctx.tag_refine(Q, 1e300, -1.0, 2, tags, ind)
    e = ind.max(dim=1).values.cpu().numpy()
    return float(np.percentile(e, 90)), float(np.percentile(e, 40))


def network(ctx, Q, flat=False):
    """A network with input normalisation from the initial leaves; flat: zero output layer, so that
    every class has probability 1/3 and no prediction is confident."""
    net = LearnedIndicator(seed=3)
    HM = torch.empty((ctx.n_patches, 4, 729), dtype=torch.float64, device="cuda")
    ctx.constraints(Q, HM)
    net.fit_normalisation(ctx.features(Q, HM))
    if flat:
        o3 = ccz4.MLP_NH * ccz4.MLP_NIN + ccz4.MLP_NH + ccz4.MLP_NH * ccz4.MLP_NH + ccz4.MLP_NH
        net.params[o3:] = 0.0
    return net


def test_unconfident_indicator_is_the_plain_criterion():
    w = workload()
    ctx, Q = start(w)
    th = thresholds(ctx, Q)
    net = network(ctx, Q, flat=True)
    c1, Q1, log1 = dynamic.evolve(ctx, Q, w, 4, 2, th[0], th[1], 2)
    ctx, Q = start(w)
    seen = []
    c2, Q2, log2 = dynamic.evolve(ctx, Q, w, 4, 2, th[0], th[1], 2, indicator=net, conf=1.0,
                                  on_tags=lambda rec, *a: seen.append(rec["step"]))
    assert seen == [2]
    assert [r["plain_refine"] for r in log1["regrids"]] == [r["plain_refine"] for r in log2["regrids"]]
    assert all(r["learned_refine"] == r["plain_refine"] for r in log2["regrids"])
    assert np.array_equal(c1.ids, c2.ids)
    assert torch.equal(Q1, Q2)
    assert log1["regrids"][0]["leaves_after"] != log1["regrids"][0]["leaves_before"]  # the mesh did change


def test_confident_indicator_keeps_plain_refine_and_adds_its_own():
    w = workload()
    ctx, Q = start(w)
    th = thresholds(ctx, Q)
    net = network(ctx, Q)
    rec_tags = []

    def on_tags(rec, ctx_, Q_, plain, feat):
        logits = net.forward(feat)
        comb = ctx_.tag_learned(logits, plain, 0.0, 2)
        own = (torch.argmax(logits, dim=1) - 1).to(torch.int8)
        rec_tags.append((plain.cpu().numpy(), comb.cpu().numpy(), own.cpu().numpy(), ctx_.ids[:, 0].copy()))

    c, Qf, log = dynamic.evolve(ctx, Q, w, 4, 2, th[0], th[1], 2, indicator=net, conf=0.0, on_tags=on_tags)
    assert len(rec_tags) == 1
    plain, comb, own, lev = rec_tags[0]
    assert np.all(comb[plain == 1] == 1)  # the plain criterion's REFINE tags stay
    # confident REFINE below max_level is added
    assert np.all(comb[(own == 1) & (lev < 2)] == 1)
    assert log["regrids"][0]["learned_refine"] == int((comb == 1).sum()) >= log["regrids"][0]["plain_refine"]
    norms, st = c.constraints(Qf)
    assert norms[2] == 0 and st == 0

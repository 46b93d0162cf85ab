"""GPU parity of the learned refinement indicator against the oracle: features, forward pass,
loss gradient, Adam step and the combination with the plain criterion.

Tolerances.  Features are FP64 stencil maxima written as FP32 log10 values: within a few FP32
ulps.  The perceptron uses the same BF16 operands on both sides (the standardised inputs are
formed in FP32 identically); what differs is the accumulation (FP32 on the matrix cores, FP64
in the oracle), which occasionally flips the BF16 rounding of a hidden activation or of a
back-propagated gradient by one BF16 ulp (2^-8 relative); the normwise bounds below allow for
a few such flips per tensor.  The layer-wise test removes that cascade by handing the oracle the
GPU's own operands of each layer (the gradient trace), and holds every gradient to 1e-4.  Adam is FP32 against FP64 with the same FP32 hyper-parameters: a
few FP32 roundings of the terms of each update.  The tags are integers: bit-exact."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle as orc  # noqa: E402
from gpu_helpers import to_gpu  # noqa: E402
from paper_2406_11626_amd import ccz4, scenarios  # noqa: E402
from paper_2406_11626_amd.learned import LearnedIndicator  # noqa: E402
from seeded_inputs import box_centers, smooth_state  # noqa: E402

NP = ccz4.MLP_NPARAM
BLOCKS = {"W1": (0, 5184), "b1": (5184, 5248), "W2": (5248, 9344), "b2": (9344, 9408), "W3": (9408, 9600),
          "b3": (9600, 9603)}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ccz4.lib()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def mlp_inputs(n, seed):
    rng = np.random.default_rng(seed)
    prm = (rng.normal(size=NP) * 0.2).astype(np.float32)
    feat = (rng.normal(size=(n, 81)) * 2.0 - 3.0).astype(np.float32)
    norm = np.concatenate([rng.normal(size=81) - 3.0, 0.3 + rng.random(81)]).astype(np.float32)
    tags = rng.integers(-1, 2, n).astype(np.int8)
    return prm, feat, norm, tags


def dev(a):
    return torch.tensor(a, device="cuda")


def test_features_parity():
    w = scenarios.config(2)
    refined = [(0, 1, 1, 1)]
    ctx = ccz4.Context((3, 3, 3), (-9.0,) * 3, (18.0,) * 3, w.bc, w.params(), refined)
    m = orc.Mesh((3, 3, 3), (-9.0,) * 3, (18.0,) * 3, w.bc, refined)
    Qo = m.zeros()
    m.init(Qo, w.scenario, w.scen)
    for p in range(m.np):  # a seeded smooth perturbation so that every feature is non-trivial
        Qo[p] += 1e-3 * smooth_state(box_centers(m.geom[p, :3], m.geom[p, 3:]), 70 + p % 5)
    m.fill_halos(Qo)
    fo = m.features(Qo)
    Qd = to_gpu(Qo)
    HM = torch.empty((ctx.n_patches, 4, 729), dtype=torch.float64, device="cuda")
    ctx.constraints(Qd, HM)
    fd = ctx.features(Qd, HM).cpu().numpy()
    assert np.isfinite(fd).all()
    err = np.abs(fd - fo)
    assert err.max() <= 4 * np.finfo(np.float32).eps * max(1.0, np.abs(fo).max()), err.max()


@pytest.mark.parametrize("n", [1, 200])
def test_forward_parity(n):
    prm, feat, norm, _ = mlp_inputs(n, 10 + n)
    logits = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    ccz4.ccz4_mlp_forward(dev(prm), dev(norm), dev(feat), n, logits)
    x = orc.mlp_standardize(feat, norm)
    zo = orc.mlp_forward(x, prm.astype(np.float64), bf16=True)[2]
    assert rel(logits.cpu().numpy(), zo) <= 2e-3, rel(logits.cpu().numpy(), zo)


def test_empty_batch():
    """No rows: the forward pass writes nothing and needs no workspace; a gradient over no rows
    (a mean over an empty set) is refused."""
    prm, feat, norm, tags = mlp_inputs(64, 7)
    logits = torch.full((1, 3), 5.0, dtype=torch.float32, device="cuda")
    ccz4.ccz4_mlp_forward(dev(prm), dev(norm), dev(feat), 0, logits)
    torch.cuda.synchronize()
    assert torch.all(logits == 5.0)
    assert ccz4.ccz4_mlp_workspace(0) == 0
    work = torch.empty(ccz4.ccz4_mlp_workspace(64), dtype=torch.float32, device="cuda")
    grad = torch.empty(ccz4.MLP_NPARAM, dtype=torch.float32, device="cuda")
    with pytest.raises(ccz4.CCZ4Error):
        ccz4.ccz4_mlp_grad(dev(prm), dev(norm), dev(feat), dev(tags), 0, work, grad)


@pytest.mark.parametrize("n", [64, 331])
def test_gradient_parity(n):
    prm, feat, norm, tags = mlp_inputs(n, 20 + n)
    ind = LearnedIndicator()
    ind.params = dev(prm)
    ind.norm = dev(norm)
    g = ind.gradient(dev(feat), dev(tags)).cpu().numpy()
    loss = float(ind.loss.item())
    x = orc.mlp_standardize(feat, norm)
    lo, go = orc.mlp_loss_grad(x, tags.astype(np.int32) + 1, prm.astype(np.float64), bf16=True)
    assert abs(loss - lo) <= 1e-4 * abs(lo), (loss, lo)
    for name, (a, b) in BLOCKS.items():
        assert rel(g[a:b], go[a:b]) <= 1e-2, (name, rel(g[a:b], go[a:b]))
    # the workspace query and its check
    with pytest.raises(ccz4.CCZ4Error):
        ccz4.ccz4_mlp_grad(ind.params, ind.norm, dev(feat), dev(tags), n, ind._work[:10], ind.grad)


@pytest.mark.parametrize("n", [64, 331])
def test_gradient_layerwise_parity(n):
    """Each layer of the GPU's forward and backward pass against the oracle's layer evaluated on
    the GPU's own operands of that layer (the trace of ccz4_mlp_grad), so that a BF16 rounding
    flip in one layer cannot propagate into the next: weight and bias gradients and the
    back-propagated pre-activation gradients to 1e-4 normwise (FP32 against FP64 accumulation),
    the BF16 activations to their own rounding."""
    prm, feat, norm, tags = mlp_inputs(n, 50 + n)
    base = ccz4.ccz4_mlp_workspace(n)
    work = torch.zeros(base + ccz4.MLP_TRACE * n, dtype=torch.float32, device="cuda")
    grad = torch.zeros(NP, dtype=torch.float32, device="cuda")
    ccz4.ccz4_mlp_grad(dev(prm), dev(norm), dev(feat), dev(tags), n, work, grad)
    g = grad.cpu().numpy().astype(np.float64)
    tr = work[base:].cpu().numpy().astype(np.float64).reshape(n, ccz4.MLP_TRACE)
    x, a1, a2 = tr[:, :81], tr[:, 81:145], tr[:, 145:209]
    d3, d2, d1 = tr[:, 209:212], tr[:, 212:276], tr[:, 276:340]
    # the BF16 input is the standardised feature rounded as the oracle rounds it
    assert np.array_equal(x, orc.bf16_array(orc.mlp_standardize(feat, norm)))
    r = orc.mlp_layers(prm.astype(np.float64), x, a1, a2, tags.astype(np.int64) + 1, d3, d2, d1)
    for name, (a, b) in BLOCKS.items():
        assert rel(g[a:b], r["g" + name].ravel()) <= 1e-4, (name, rel(g[a:b], r["g" + name].ravel()))
    for name, got in (("d3", d3), ("d2", d2), ("d1", d1)):
        assert rel(got, r[name]) <= 1e-4, (name, rel(got, r[name]))
    # activations: the BF16 rounding (half a unit in the last place, 2^-8 relative at most) of
    # ReLU of the pre-activation, up to the FP32 accumulation of the matrix cores
    for got, z in ((a1, r["z1"]), (a2, r["z2"])):
        ref = np.maximum(z, 0.0)
        assert np.all(np.abs(got - ref) <= 2.0 ** -8 * ref + 1e-5 * np.abs(z).max())
        flip = (got > 0) != (ref > 0)  # ReLU masks differ only where z is at rounding level
        assert np.all(np.abs(z[flip]) <= 1e-5 * np.abs(z).max())
    # the plain workspace gives the same gradient without the trace
    g2 = torch.zeros(NP, dtype=torch.float32, device="cuda")
    ccz4.ccz4_mlp_grad(dev(prm), dev(norm), dev(feat), dev(tags), n, work[:base], g2)
    assert torch.equal(g2, grad)


def test_adam_parity():
    rng = np.random.default_rng(30)
    p = rng.normal(size=NP).astype(np.float32)
    m = (rng.normal(size=NP) * 0.1).astype(np.float32)
    v = (rng.random(NP) * 0.01).astype(np.float32)
    g = rng.normal(size=NP).astype(np.float32)
    pd, md, vd = dev(p), dev(m), dev(v)
    ccz4.ccz4_mlp_adam(pd, md, vd, dev(g), 3, 1e-3)
    po, mo, vo = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    # the kernel holds lr, beta1, beta2 and eps in FP32: the oracle takes the same values
    f32 = lambda a: float(np.float32(a))  # noqa: E731
    orc.adam_step(po, mo, vo, g.astype(np.float64), 3, f32(1e-3), f32(0.9), f32(0.999), f32(1e-8))
    # FP32 against FP64: a few roundings relative to the size of the terms of each update
    eps32 = np.finfo(np.float32).eps
    bm = 4 * eps32 * (0.9 * np.abs(m) + 0.1 * np.abs(g))
    bv = 4 * eps32 * (0.999 * v + 0.001 * g.astype(np.float64) ** 2)
    assert np.all(np.abs(md.cpu().numpy() - mo) <= bm)
    assert np.all(np.abs(vd.cpu().numpy() - vo) <= bv)
    step = np.abs(po - p)  # the change of the parameters is accurate to FP32 relative rounding
    assert np.all(np.abs(pd.cpu().numpy() - po) <= 1e-5 * step + 2 * eps32 * np.abs(p))
    with pytest.raises(ccz4.CCZ4Error):
        ccz4.ccz4_mlp_adam(pd, md, vd, dev(g), 0, 1e-3)


def test_tag_learned_parity():
    w = scenarios.config(2)
    refined = [(0, 1, 1, 1), (1, 4, 4, 4)]
    ctx = ccz4.Context((3, 3, 3), (-9.0,) * 3, (18.0,) * 3, w.bc, w.params(), refined)
    m = orc.Mesh((3, 3, 3), (-9.0,) * 3, (18.0,) * 3, w.bc, refined)
    rng = np.random.default_rng(40)
    for trial in range(4):
        logits = (rng.normal(size=(m.np, 3)) * (1 + 3 * trial)).astype(np.float32)
        plain = rng.integers(-1, 2, m.np).astype(np.int8)
        if trial == 3:  # whole families asked to coarsen, so that the family rule is exercised
            plain[m.ids[:, 0] == 2] = -1
        for conf in (0.0, 0.6, 0.95):
            for max_level in (1, 3):
                got = ctx.tag_learned(dev(logits), dev(plain), conf, max_level).cpu().numpy()
                assert np.array_equal(got, m.tag_learned(logits, plain, conf, max_level)), (trial, conf, max_level)

"""Pins of the learned-indicator oracle (oracle/ccz4_mlp.c) against facts that do not come from
the oracle itself: BF16 rounding against torch's float32 -> bfloat16 conversion, the loss
gradient against central finite differences, closed forms at zero weights and for Adam with a
constant gradient, exact invariance under a permutation of the hidden units, the features of
fields whose FD4 gradients are exact, and the combination rule on hand-made cases."""
import numpy as np
import pytest

import oracle as orc
from seeded_inputs import box_centers

torch = pytest.importorskip("torch")

NP = orc.MLP_NPARAM
OW1, OB1 = 0, 64 * 81
OW2, OB2 = OB1 + 64, OB1 + 64 + 64 * 64
OW3, OB3 = OB2 + 64, OB2 + 64 + 3 * 64


def rand_params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(size=NP) * scale


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    vals = np.concatenate([
        rng.normal(size=4000) * 10.0 ** rng.integers(-30, 30, 4000),
        # exact ties between two BF16 neighbours, both parities of the kept bit
        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 2.0 ** -130 * 1.5, 3.0e38, 0.0, -0.0],
    ]).astype(np.float32)
    ref = torch.tensor(vals).to(torch.bfloat16).to(torch.float32).numpy()
    got = np.array([orc.bf16_round(float(v)) for v in vals], dtype=np.float32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("seed", [1, 2])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    prm = rand_params(seed)
    x = rng.normal(size=(7, 81))
    lab = rng.integers(0, 3, 7)
    loss, g = orc.mlp_loss_grad(x, lab, prm, bf16=False)
    idx = np.concatenate([rng.choice(NP, 90, replace=False), np.arange(OB3, NP), np.arange(OB1, OB1 + 4)])
    h = 1e-5
    fd = np.zeros(idx.size)
    for n, q in enumerate(idx):
        pp, pm = prm.copy(), prm.copy()
        pp[q] += h
        pm[q] -= h
        fd[n] = (orc.mlp_loss_grad(x, lab, pp, False)[0] - orc.mlp_loss_grad(x, lab, pm, False)[0]) / (2 * h)
    assert np.linalg.norm(fd - g[idx]) <= 1e-6 * np.linalg.norm(g[idx])
    # the loss is the mean cross-entropy of the forward logits
    z = orc.mlp_forward(x, prm, bf16=False)[2]
    ce = -np.mean(z[np.arange(7), lab] - np.log(np.exp(z).sum(axis=1)))
    assert abs(ce - loss) < 1e-12


def test_zero_weights_closed_form():
    prm = np.zeros(NP)
    rng = np.random.default_rng(3)
    x = rng.normal(size=(5, 81))
    lab = np.array([0, 1, 2, 2, 1])
    for bf16 in (False, True):
        loss, g = orc.mlp_loss_grad(x, lab, prm, bf16)
        assert abs(loss - np.log(3.0)) < 1e-15
        onehot = np.eye(3)[lab]
        assert np.allclose(g[OB3:], np.mean(1.0 / 3.0 - onehot, axis=0), atol=1e-16)
        assert np.all(g[:OB3] == 0.0)


@pytest.mark.parametrize("bf16", [False, True])
def test_hidden_unit_permutation_invariance(bf16):
    rng = np.random.default_rng(4)
    prm = rand_params(4)
    x = rng.normal(size=(6, 81))
    W1 = prm[OW1:OB1].reshape(64, 81)
    b1 = prm[OB1:OW2]
    W2 = prm[OW2:OB2].reshape(64, 64)
    b2 = prm[OB2:OW3]
    W3 = prm[OW3:OB3].reshape(3, 64)
    p1, p2 = rng.permutation(64), rng.permutation(64)
    q = np.concatenate([W1[p1].ravel(), b1[p1], W2[p2][:, p1].ravel(), b2[p2], W3[:, p2].ravel(), prm[OB3:]])
    z = orc.mlp_forward(x, prm, bf16)[2]
    zq = orc.mlp_forward(x, q, bf16)[2]
    assert np.allclose(z, zq, rtol=1e-13, atol=1e-13)


def test_adam_constant_gradient_closed_form():
    rng = np.random.default_rng(5)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    lr, eps = 1e-2, 1e-8
    for t in range(1, 8):
        orc.adam_step(p, m, v, g, t, lr, 0.9, 0.999, eps)
    # with a constant gradient the bias-corrected moments are exactly g and g^2
    assert np.allclose(p, p0 - 7 * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-12)


def test_features_of_fields_with_exact_stencils():
    """phi and alpha linear in x, y, z on one patch: FD4 of chi = phi^2 and of alpha are exact,
    so the block maxima of dx |grad chi| and dx |grad alpha| have closed forms; the dx^2 |H|
    block maxima are those of the (separately pinned) constraint fields."""
    m = orc.Mesh((1, 1, 1), (0.0, 0.0, 0.0), (0.9, 0.9, 0.9), 0)
    Q = m.zeros()
    org, dx = m.geom[0, :3], m.geom[0, 3:]
    P = box_centers(org, dx)  # (15, 15, 15, 3) cell centres of the whole box, [z][y][x]
    a = np.array([0.3, -0.2, 0.5])
    b = np.array([-0.4, 0.1, 0.25])
    phi = 1.2 + P @ a
    alpha = 0.8 + P @ b
    Q[0, ..., 0] = Q[0, ..., 3] = Q[0, ..., 5] = 1.0
    Q[0, ..., 10] = phi
    Q[0, ..., 6] = alpha
    f = m.features(Q)[0].reshape(27, 3)
    _, HM = m.constraints(Q, want_fields=True)
    H = np.abs(HM[0, :, 0]).reshape(9, 9, 9)
    h = dx[0]
    gchi = h * 2.0 * np.abs(phi[3:12, 3:12, 3:12]) * np.linalg.norm(a)
    for bz in range(3):
        for by in range(3):
            for bx in range(3):
                blk = (slice(3 * bz, 3 * bz + 3), slice(3 * by, 3 * by + 3), slice(3 * bx, 3 * bx + 3))
                n = (bz * 3 + by) * 3 + bx
                assert abs(f[n, 0] - np.log10(gchi[blk].max() + 1e-12)) < 1e-12
                assert abs(f[n, 1] - np.log10(h * np.linalg.norm(b) + 1e-12)) < 1e-12
                assert abs(f[n, 2] - np.log10(h * h * H[blk].max() + 1e-12)) < 1e-12


def test_learned_tag_rule_cases():
    """One level-0 cube refined into 27 level-1 leaves plus 7 level-0 leaves; hand-made logits."""
    m = orc.Mesh((2, 2, 2), (0, 0, 0), (2.0, 2.0, 2.0), 0, [(0, 0, 0, 0)])
    lev = m.ids[:, 0]
    l0 = np.where(lev == 0)[0]
    l1 = np.where(lev == 1)[0]
    sure_ref = [0.0, 0.0, 9.0]
    sure_keep = [0.0, 9.0, 0.0]
    sure_coarse = [9.0, 0.0, 0.0]
    unsure = [0.0, 0.0, 0.1]
    n = m.np
    # plain REFINE stays whatever the network says; a confident REFINE is added below max_level
    logits = np.tile(sure_keep, (n, 1))
    plain = np.zeros(n, np.int8)
    plain[l0[0]] = 1
    logits[l0[1]] = sure_ref
    logits[l0[2]] = unsure
    logits[l1[0]] = sure_ref
    t = m.tag_learned(logits, plain, 0.9, 1)
    assert t[l0[0]] == 1 and t[l0[1]] == 1 and t[l0[2]] == 0
    assert t[l1[0]] == 0  # level 1 is max_level: no refinement
    assert m.tag_learned(logits, plain, 0.9, 2)[l1[0]] == 1
    # a plain COARSEN of the whole family survives when the network agrees or is unsure ...
    plain = np.zeros(n, np.int8)
    plain[l1] = -1
    logits = np.tile(sure_coarse, (n, 1))
    logits[l1[:5]] = unsure
    t = m.tag_learned(logits, plain, 0.9, 2)
    assert np.all(t[l1] == -1) and np.all(t[l0] == 0)
    # ... and one confident KEEP vetoes it for the whole family
    logits[l1[7]] = sure_keep
    t = m.tag_learned(logits, plain, 0.9, 2)
    assert np.all(t[l1] == 0)
    # arg-max ties go to the higher class
    logits = np.tile([1.0, 1.0, 1.0], (n, 1))
    plain = np.zeros(n, np.int8)
    assert np.all(m.tag_learned(logits, plain, 0.3, 2)[l0] == 1)


@pytest.mark.parametrize("bf16", [False, True])
def test_layerwise_form_chains_to_the_loss_gradient(bf16):
    """The layer-by-layer form of the oracle, chained on its own outputs (activations ReLU of the
    pre-activations, rounded to BF16 where the matrix cores take them), reproduces the whole
    loss gradient of the oracle, which the finite-difference test above pins."""
    rng = np.random.default_rng(7)
    n = 37
    prm = rand_params(8)
    x = rng.normal(size=(n, 81))
    if bf16:
        x = orc.bf16_array(x)
    labels = rng.integers(0, 3, n)
    rnd = orc.bf16_array if bf16 else (lambda a: a)
    z = np.zeros((n, 64))
    d = np.zeros((n, 3))
    a1 = rnd(np.maximum(orc.mlp_layers(prm, x, z, z, labels, d, z, z, bf16)["z1"], 0.0))
    a2 = rnd(np.maximum(orc.mlp_layers(prm, x, a1, z, labels, d, z, z, bf16)["z2"], 0.0))
    d3 = orc.mlp_layers(prm, x, a1, a2, labels, d, z, z, bf16)["d3"]
    d2 = orc.mlp_layers(prm, x, a1, a2, labels, d3, z, z, bf16)["d2"]
    d1 = orc.mlp_layers(prm, x, a1, a2, labels, d3, d2, z, bf16)["d1"]
    r = orc.mlp_layers(prm, x, a1, a2, labels, d3, d2, d1, bf16)
    g = np.concatenate([r["gW1"].ravel(), r["gb1"], r["gW2"].ravel(), r["gb2"], r["gW3"].ravel(), r["gb3"]])
    _, go = orc.mlp_loss_grad(x, labels, prm, bf16=bf16)
    np.testing.assert_allclose(g, go, rtol=1e-12, atol=1e-14 * np.abs(go).max())
    # and the logits of the chained form are the oracle's forward pass
    np.testing.assert_allclose(r["z3"], orc.mlp_forward(x, prm, bf16=bf16)[2], rtol=1e-12, atol=1e-14)

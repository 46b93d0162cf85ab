"""Learned refinement indicator: training data from the solver's own runs, training and use.

The indicator is a small perceptron on per-leaf field statistics (``ccz4_features``) that
predicts the tag the plain criterion will give a leaf some steps ahead, so that refinement can
be placed before a moving feature (the outgoing gauge pulse, a drifting puncture) arrives; the
plain criterion stays in charge (``ccz4_tag_learned``: its REFINE tags are kept and it is the
fallback when the network is not confident).  Inference, loss, gradient and the Adam update run
in the library's kernels; this module only moves buffers.
"""
import numpy as np

from . import ccz4


class LearnedIndicator:
    """Device-resident parameters (FP32 master weights, Adam moments, input normalisation)."""

    def __init__(self, seed=0):
        import torch
        rng = np.random.default_rng(seed)
        prm = np.zeros(ccz4.MLP_NPARAM, dtype=np.float32)
        o = 0
        for fan_out, fan_in in ((ccz4.MLP_NH, ccz4.MLP_NIN), (ccz4.MLP_NH, ccz4.MLP_NH), (ccz4.MLP_NOUT, ccz4.MLP_NH)):
            prm[o:o + fan_out * fan_in] = rng.normal(size=fan_out * fan_in) * np.sqrt(2.0 / fan_in)  # He
            o += fan_out * fan_in + fan_out  # biases start at zero
        self.params = torch.tensor(prm, device="cuda")
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.norm = torch.tensor(np.concatenate([np.zeros(ccz4.MLP_NIN), np.ones(ccz4.MLP_NIN)]),
                                 dtype=torch.float32, device="cuda")
        self.step = 0
        self._work = None

    def fit_normalisation(self, feat):
        """mu and 1/sigma per feature (host statistics of an (n, 81) device tensor)."""
        import torch
        f = feat.cpu().numpy().astype(np.float64)
        mu = f.mean(axis=0)
        sd = np.maximum(f.std(axis=0), 1e-3)
        self.norm = torch.tensor(np.concatenate([mu, 1.0 / sd]), dtype=torch.float32, device="cuda")

    def forward(self, feat, stream=None):
        import torch
        n = feat.shape[0]
        logits = torch.empty((n, ccz4.MLP_NOUT), dtype=torch.float32, device="cuda")
        ccz4.ccz4_mlp_forward(self.params, self.norm, feat, n, logits, stream)
        return logits

    def gradient(self, feat, tags, stream=None):
        import torch
        n = feat.shape[0]
        need = ccz4.ccz4_mlp_workspace(n)
        if self._work is None or self._work.numel() < need:
            self._work = torch.empty(need, dtype=torch.float32, device="cuda")
        ccz4.ccz4_mlp_grad(self.params, self.norm, feat, tags, n, self._work, self.grad, self.loss, stream)
        return self.grad

    def train(self, feat, tags, iters, lr=3e-3, stream=None):
        """Full-batch Adam on (feat, tags); returns the loss after the last step."""
        for _ in range(iters):
            self.gradient(feat, tags, stream)
            self.step += 1
            ccz4.ccz4_mlp_adam(self.params, self.m, self.v, self.grad, self.step, lr, stream=stream)
        self.gradient(feat, tags, stream)
        return float(self.loss.item())


def snapshots(ctx, Q, dt, steps, every, theta_r, theta_c, max_level, bufs=None):
    """Evolve Q (halos filled on entry) for `steps` RK4 steps; every `every` steps (and at t = 0)
    record the leaf features and the plain criterion's tags.  Returns [(feat, tags)] on device."""
    import torch
    if bufs is None:
        bufs = tuple(ctx.new_state(0.0) for _ in range(3))
    HM = torch.empty((ctx.n_patches, 4, 729), dtype=torch.float64, device="cuda")
    out = []
    tags = torch.empty(ctx.n_patches, dtype=torch.int8, device="cuda")
    for s in range(steps + 1):
        if s % every == 0:
            ctx.constraints(Q, HM)
            feat = ctx.features(Q, HM)
            ctx.tag_refine(Q, theta_r, theta_c, max_level, tags)
            out.append((feat.clone(), tags.clone()))
        if s < steps:
            ctx.rk4_step_fused(Q, dt, bufs)
    return out


def miss_rate(predicted, truth):
    """Fraction of the leaves tagged REFINE in `truth` that `predicted` does not tag REFINE,
    and the number of REFINE tags of `predicted` that `truth` does not have."""
    p = predicted.cpu().numpy()
    t = truth.cpu().numpy()
    need = t == 1
    miss = float(np.sum(need & (p != 1))) / max(1, int(np.sum(need)))
    extra = int(np.sum((p == 1) & ~need))
    return miss, extra


def anticipation(ind, ctx, snaps, conf=0.6, max_level=2):
    """Score of the indicator on consecutive snapshots [(feat, plain tags)]: for each pair (k, k+1)
    the tags at k are used as the prediction of the plain tags at k+1.  Returns the mean over
    pairs of (miss rate, extra REFINE tags) for the plain criterion alone, for the combination
    with the network (ccz4_tag_learned) and for the network's arg-max alone."""
    import torch
    out = {"plain": [], "combined": [], "network": []}
    for k in range(len(snaps) - 1):
        feat, plain = snaps[k]
        truth = snaps[k + 1][1]
        logits = ind.forward(feat)
        comb = ctx.tag_learned(logits, plain, conf, max_level)
        net = (torch.argmax(logits, dim=1) - 1).to(torch.int8)
        out["plain"].append(miss_rate(plain, truth))
        out["combined"].append(miss_rate(comb, truth))
        out["network"].append(miss_rate(net, truth))
    return {k: tuple(np.mean(np.array(v, dtype=np.float64), axis=0)) for k, v in out.items()}

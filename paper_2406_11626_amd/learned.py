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


def face_neighbours(ids, n0, periodic=False):
    """Leaves sharing a face with each leaf of a 2:1-balanced forest (ids: (n, 4) rows of level,
    i, j, k; n0: the level-0 cube counts): across each face, the leaf of the same level, else the
    coarser leaf that contains that cube, else the finer leaves that touch the face.  A list of
    index arrays."""
    index = {tuple(int(v) for v in r): p for p, r in enumerate(ids)}
    out = []
    for me, (lev, i, j, k) in enumerate(tuple(int(v) for v in r) for r in ids):
        size = [n0[a] * 3 ** lev for a in range(3)]
        nb = set()
        for a in range(3):
            for side in (-1, 1):
                c = [i, j, k]
                c[a] += side
                if not 0 <= c[a] < size[a]:
                    if not periodic:
                        continue
                    c[a] %= size[a]
                q = index.get((lev, *c))
                if q is None and lev > 0:
                    q = index.get((lev - 1, c[0] // 3, c[1] // 3, c[2] // 3))
                if q is not None:
                    if q != me:  # a periodic axis of one cube wraps onto the leaf itself
                        nb.add(q)
                    continue
                others = [b for b in range(3) if b != a]
                for u in range(3):  # the nine finer leaves across the face
                    for v in range(3):
                        f = [3 * c[0], 3 * c[1], 3 * c[2]]
                        f[a] += 0 if side > 0 else 2
                        f[others[0]] += u
                        f[others[1]] += v
                        q = index.get((lev + 1, *f))
                        if q is not None:
                            nb.add(q)
        out.append(np.array(sorted(nb), dtype=np.int64))
    return out


def adjacent_fallback(comb, plain, neighbours):
    """The combination with the plain criterion deciding on every leaf that shares a face with a
    leaf it tags REFINE (the network's additions there are dropped)."""
    c = comb.cpu().numpy().copy()
    pl = plain.cpu().numpy()
    near = np.array([bool(np.any(pl[nb] == 1)) if len(nb) else False for nb in neighbours])
    c[near] = pl[near]
    return c


def anticipation(ind, ctx, snaps, conf=0.6, max_level=2):
    """Score of the indicator on consecutive snapshots [(feat, plain tags)]: for each pair (k, k+1)
    the tags at k are used as the prediction of the plain tags at k+1.  Returns the mean over
    pairs of (miss rate, extra REFINE tags) for the plain criterion alone, for the combination
    with the network (ccz4_tag_learned), for that combination with the plain criterion deciding
    on every leaf next to a plain REFINE, and for the network's arg-max alone."""
    import torch
    out = {"plain": [], "combined": [], "combined_adjacent_fallback": [], "network": []}
    neighbours = face_neighbours(ctx.ids, ctx.n0, ctx.bc == ccz4.BC_PERIODIC)
    for k in range(len(snaps) - 1):
        feat, plain = snaps[k]
        truth = snaps[k + 1][1]
        logits = ind.forward(feat)
        comb = ctx.tag_learned(logits, plain, conf, max_level)
        net = (torch.argmax(logits, dim=1) - 1).to(torch.int8)
        out["plain"].append(miss_rate(plain, truth))
        out["combined"].append(miss_rate(comb, truth))
        out["combined_adjacent_fallback"].append(
            miss_rate(torch.from_numpy(adjacent_fallback(comb, plain, neighbours)), truth))
        out["network"].append(miss_rate(net, truth))
    return {k: tuple(np.mean(np.array(v, dtype=np.float64), axis=0)) for k, v in out.items()}

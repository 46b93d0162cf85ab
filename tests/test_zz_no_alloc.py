"""ccz4_mlp_grad_noalloc (the gradient entry point that allocates nothing, its per-tile partials in
the library's per-GPU array) against ccz4_mlp_grad with a caller workspace: the same kernels and
the same reduction order, so the gradients and losses agree bit for bit, on two calls in a row
(the second with fewer rows, so that the array holds stale partials of the first beyond the
second's tiles), and it rejects more rows than the array holds."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2406_11626_amd import ccz4  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ccz4.lib()


def inputs(n, seed):
    rng = np.random.default_rng(seed)
    dev = lambda a: torch.tensor(a, device="cuda")  # noqa: E731
    prm = (rng.normal(size=ccz4.MLP_NPARAM) * 0.2).astype(np.float32)
    feat = (rng.normal(size=(n, 81)) * 2.0 - 3.0).astype(np.float32)
    norm = np.concatenate([rng.normal(size=81) - 3.0, 0.3 + rng.random(81)]).astype(np.float32)
    tags = rng.integers(-1, 2, n).astype(np.int8)
    return dev(prm), dev(norm), dev(feat), dev(tags)


def with_workspace(prm, norm, feat, tags, n):
    work = torch.empty(ccz4.ccz4_mlp_workspace(n), dtype=torch.float32, device="cuda")
    g = torch.empty(ccz4.MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    ccz4.ccz4_mlp_grad(prm, norm, feat, tags, n, work, g, loss)
    return g, loss


def without(prm, norm, feat, tags, n):
    g = torch.full((ccz4.MLP_NPARAM,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
    ccz4.ccz4_mlp_grad_noalloc(prm, norm, feat, tags, n, g, loss)
    return g, loss


def test_noalloc_gradient_equals_workspace_gradient():
    for n, seed in ((ccz4.MLP_NOALLOC_MAX_ROWS, 1), (331, 2), (1, 3)):
        args = inputs(n, seed)
        g0, l0 = with_workspace(*args, n)
        g1, l1 = without(*args, n)
        torch.cuda.synchronize()
        assert torch.equal(g1, g0), n
        assert torch.equal(l1, l0), n
        assert torch.isfinite(g1).all()


def test_noalloc_rejects_too_many_rows():
    n = ccz4.MLP_NOALLOC_MAX_ROWS + 1
    args = inputs(n, 4)
    with pytest.raises(ccz4.CCZ4Error):
        without(*args, n)
    with pytest.raises(ccz4.CCZ4Error):
        without(*args, 0)

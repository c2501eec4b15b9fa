"""The gradient entry point that allocates nothing (pdf_mlp_grad_noalloc)
against pdf_mlp_grad, which takes a caller-owned workspace: loss and
gradient bit for bit, on two calls in a row, the second with a smaller batch
(the static scratch keeps the first call's partials, which the second must
not read), and the size limit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_4548_amd as P
    from paper_1003_4548_amd import mlp as PM
    P.load_library()
    return P, PM, torch


def _rows(rng, B):
    rows = np.zeros((B, 64), np.float32)
    rows[:, :32] = rng.normal(size=(B, 32))
    rows[:, 32:40] = rng.normal(size=(B, 8))
    lw = rng.random(size=(B, 8))
    lw /= lw.sum(axis=1, keepdims=True)
    lw[rng.random(B) < 0.1] = 0.0
    rows[:, 40:48] = lw
    return rows


def test_noalloc_gradient_equals_workspace_gradient(gpu):
    P, PM, torch = gpu
    print("[case] mlp gradient without workspace: batches 1000 then 37", flush=True)
    rng = np.random.default_rng(11)
    net = PM.ConditionalMeanNet(seed=5)
    big = torch.as_tensor(_rows(rng, 1000)).cuda()
    net.fit_norm(big)
    # preallocated outputs: the no-alloc calls themselves allocate nothing
    outs = [(torch.empty(1, dtype=torch.float32, device="cuda"),
             torch.empty(PM.NPARAM, dtype=torch.float32, device="cuda")) for _ in range(2)]
    for k, b in enumerate((1000, 37)):    # 37: fewer tiles than the call before, a ragged last tile
        l_ref, g_ref = net.grad(big, b)
        l_na, g_na = net.grad_noalloc(big, b, out=outs[k])
        torch.cuda.synchronize()
        assert np.isfinite(g_ref.cpu().numpy()).all()
        np.testing.assert_array_equal(l_na.cpu().numpy(), l_ref.cpu().numpy())
        np.testing.assert_array_equal(g_na.cpu().numpy(), g_ref.cpu().numpy())


def test_noalloc_rejects_batches_beyond_its_scratch(gpu):
    P, PM, torch = gpu
    print("[case] mlp gradient without workspace: size limit", flush=True)
    net = PM.ConditionalMeanNet(seed=5)
    rows = torch.zeros((PM.NOALLOC_MAX_BATCH + 1, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(P.PdfError) as ei:
        net.grad_noalloc(rows)
    assert ei.value.code == -3
    with pytest.raises(P.PdfError):
        net.grad_noalloc(rows, 0)
    l, g = net.grad_noalloc(rows, PM.NOALLOC_MAX_BATCH)   # the largest batch is accepted
    torch.cuda.synchronize()
    assert np.isfinite(g.cpu().numpy()).all()

"""The allocation-free gradient entry point (xtm_mlp_grad_noalloc, for
callers that cannot allocate device memory) against xtm_mlp_grad with a
caller-provided workspace: same kernels, so bitwise equal, on consecutive
calls that reuse the library's fixed workspace with a smaller batch after a
larger one."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_00317_amd as P
    P.lib()
    return P


def _inputs(B, seed):
    rng = np.random.default_rng(seed)
    sizes = [(16, 128), (128,), (128, 128), (128,), (128,), (1,)]
    parts = []
    for k, shape in enumerate(sizes):
        n = int(np.prod(shape))
        std = math.sqrt(2.0 / shape[0]) if k in (0, 2, 4) else 0.05
        parts.append(rng.normal(0, std, n))
    theta = np.concatenate(parts).astype(np.float32)
    x = (rng.normal(size=(B, 16)) * np.linspace(0.5, 3, 16) + np.linspace(-2, 2, 16)).astype(np.float32)
    norm = np.concatenate([np.linspace(-2, 2, 16), 1 / np.linspace(0.5, 3, 16)]).astype(np.float32)
    y = (rng.random(B) < 0.3).astype(np.float32)
    return theta, x, norm, y


def test_noalloc_gradient_equals_workspace_gradient(P):
    import torch
    assert P.MLP_PARAMS == 18817
    dev = "cuda"
    grad = torch.empty(P.MLP_PARAMS, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    # a full batch, then smaller ones with ragged tails (the fixed workspace
    # keeps the earlier call's partials beyond the new batch's blocks)
    for B, seed in ((4096, 11), (1000, 12), (1, 13)):
        theta, x, norm, y = _inputs(B, seed)
        t = lambda a: torch.tensor(a, device=dev)
        th, nm, X, Y = t(theta), t(norm), t(x), t(y)
        w = float((y == 0).sum() / max((y == 1).sum(), 1))
        grad.fill_(float("nan"))
        loss.fill_(float("nan"))
        print(f"[no-alloc] B={B} seed={seed}", flush=True)
        P.mlp_grad_noalloc(th, nm, X, Y, w, grad, loss)
        g_ref, l_ref = P.mlp_grad(th, nm, X, Y, w)
        torch.cuda.synchronize()
        a = grad.cpu().numpy().view(np.uint32)
        b = g_ref.cpu().numpy().view(np.uint32)
        assert np.isfinite(grad.cpu().numpy()).all()
        assert np.array_equal(a, b), (B, int(np.sum(a != b)))
        assert loss.cpu().numpy().view(np.uint32)[0] == l_ref.cpu().numpy().view(np.uint32)[0]


def test_noalloc_gradient_without_loss_output(P):
    import torch
    theta, x, norm, y = _inputs(300, 21)
    t = lambda a: torch.tensor(a, device="cuda")
    grad = torch.full((P.MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
    P.mlp_grad_noalloc(t(theta), t(norm), t(x), t(y), 2.0, grad, None)
    g_ref, _ = P.mlp_grad(t(theta), t(norm), t(x), t(y), 2.0)
    assert np.array_equal(grad.cpu().numpy().view(np.uint32), g_ref.cpu().numpy().view(np.uint32))


def test_noalloc_gradient_rejects_batches_beyond_its_workspace(P):
    import torch
    theta, x, norm, y = _inputs(P.MLP_NOALLOC_MAX_BATCH + 1, 31)
    t = lambda a: torch.tensor(a, device="cuda")
    grad = torch.empty(P.MLP_PARAMS, dtype=torch.float32, device="cuda")
    with pytest.raises(P.XtmError) as ei:
        P.mlp_grad_noalloc(t(theta), t(norm), t(x), t(y), 2.0, grad)
    assert ei.value.code == -1

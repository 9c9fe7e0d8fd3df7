"""The MLP backward entry point that allocates nothing
(dem_mlp_backward_noalloc, for callers that cannot allocate device memory)
against the entry point it mirrors (dem_mlp_backward), through the C ABI.

Both run the same kernels in the same summation order, so the gradient and
the loss must agree bit for bit.  Two calls in a row, the second with fewer
samples, check that what the shared scratch array kept from the first call
does not leak into the second; the size limit is refused with a message and
leaves the outputs untouched.
"""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

NPARAM = 1313
NF = 6


@pytest.fixture(scope="module")
def dem():
    import paper_2311_04648_amd as d
    if not os.path.exists(d.LIB_PATH):
        from paper_2311_04648_amd import build
        build.build()
    d._torch()
    return d


def _data(seed, n):
    rng = np.random.default_rng(seed)
    p = W.f32(rng.normal(0, 0.3, size=NPARAM))
    X = W.f32(rng.normal(0, 1.0, size=(n, NF)))
    T = W.f32(rng.normal(0, 1.0, size=n))
    return p, X, T


def test_noalloc_backward_equals_workspace_backward(dem):
    import torch
    dev = "cuda"
    grad = torch.empty(NPARAM, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    # largest allowed size first, then a smaller one that leaves stale
    # partials of the first call beyond its own blocks
    for n, tau, seed in [(dem.MLP_NOALLOC_MAX, 0.05, 3), (1000, 0.3, 4), (1, 0.05, 5)]:
        p, X, T = _data(seed, n)
        tp = torch.tensor(p, dtype=torch.float32, device=dev)
        tX = torch.tensor(X, dtype=torch.float32, device=dev)
        tT = torch.tensor(T, dtype=torch.float32, device=dev)
        gref, lref = dem.mlp_backward(tp, tX, tT, tau)
        grad.fill_(float("nan"))
        loss.fill_(float("nan"))
        dem.mlp_backward_noalloc(tp, tX, tT, tau, grad, loss)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(grad.cpu().numpy(), gref.cpu().numpy())
        np.testing.assert_array_equal(loss.cpu().numpy(), lref.cpu().numpy())
        assert np.isfinite(grad.cpu().numpy()).all()


def test_noalloc_backward_refuses_oversize_and_bad_args(dem):
    import torch
    dev = "cuda"
    n = dem.MLP_NOALLOC_MAX + 1
    p, X, T = _data(9, n)
    grad = torch.full((NPARAM,), 7.0, dtype=torch.float32, device=dev)
    loss = torch.full((1,), 7.0, dtype=torch.float32, device=dev)
    with pytest.raises(dem.DemError) as ei:
        dem.mlp_backward_noalloc(torch.tensor(p, dtype=torch.float32, device=dev),
                                 torch.tensor(X, dtype=torch.float32, device=dev),
                                 torch.tensor(T, dtype=torch.float32, device=dev), 0.05, grad, loss)
    assert ei.value.status == 2 and "exceeds" in str(ei.value)
    with pytest.raises(dem.DemError) as ei:
        dem.mlp_backward_noalloc(torch.tensor(p, dtype=torch.float32, device=dev),
                                 torch.tensor(X[:10], dtype=torch.float32, device=dev),
                                 torch.tensor(T[:10], dtype=torch.float32, device=dev), 1.5, grad, loss)
    assert ei.value.status == 1
    torch.cuda.synchronize()
    assert (grad.cpu().numpy() == 7.0).all() and loss.item() == 7.0

"""The allocation-free loss/gradient entry point of the rank predictor against the
workspace form, through the C ABI: two calls in a row, the second with fewer
samples, and the limit on the number of samples."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2108_12574_amd as cbd
    from paper_2108_12574_amd import _lib

DEV = "cuda:0"


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    P = cbd.lib().rank_mlp_params()
    params = torch.tensor(rng.standard_normal(P) * 0.2, dtype=torch.float32, device=DEV)
    X = torch.tensor(rng.random((n, 6)), dtype=torch.float32, device=DEV)
    t = torch.tensor(rng.random(n) * 6.0, dtype=torch.float32, device=DEV)
    return params, X, t


def _with_workspace(params, X, t):
    n = X.shape[0]
    L = cbd.lib()
    ws = torch.empty(L.rank_mlp_workspace_bytes(n), dtype=torch.uint8, device=DEV)
    g = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    assert L.rank_mlp_loss_grad(_p(params), n, _p(X), _p(t), _p(g), _p(loss), _p(ws), ws.numel(), None) == 0
    torch.cuda.synchronize()
    return g, loss


def _no_alloc(params, X, t):
    n = X.shape[0]
    g = torch.full_like(params, float("nan"))
    loss = torch.full((1,), float("nan"), dtype=torch.float32, device=DEV)
    rc = cbd.lib().rank_mlp_loss_grad_noalloc(_p(params), n, _p(X), _p(t), _p(g), _p(loss), None)
    assert rc == 0, cbd.lib().cbd_last_error()
    torch.cuda.synchronize()
    return g, loss


def test_no_alloc_matches_workspace_form_twice():
    # same kernels, same summation order: the results are identical, on a first call
    # and on a second, smaller one (which must not see the first call's scratch)
    for n, seed in [(5000, 0), (700, 1)]:
        params, X, t = _inputs(n, seed)
        g1, l1 = _with_workspace(params, X, t)
        g2, l2 = _no_alloc(params, X, t)
        assert torch.equal(g1, g2), (n, (g1 - g2).abs().max().item())
        assert torch.equal(l1, l2)
        assert torch.isfinite(g2).all()


def test_no_alloc_limit():
    L = cbd.lib()
    params, X, t = _inputs(8, 2)
    g = torch.empty_like(params)
    big = 16385
    assert L.rank_mlp_loss_grad_noalloc(_p(params), big, _p(X), _p(t), _p(g), None, None) == _lib.EARG
    assert b"exceed the limit of 16384" in L.cbd_last_error()
    assert L.rank_mlp_loss_grad_noalloc(_p(params), 0, _p(X), _p(t), _p(g), None, None) == _lib.EARG

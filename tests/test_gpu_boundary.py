"""GPU tests of the boundary's workspace contract: caller-owned factor workspace,
rank hints and ranks_out, apply column blocks, and rs_apply_sub (lemma l:subdomain,
Section 3.2, with the subproblems of (e:ai) and the sum (e:ad))."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import dd, ie, rs

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2108_12574_amd as cbd
    from paper_2108_12574_amd import _lib

DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def cfg():
    n = 64
    P = cbd.Problem(2, n, device=DEV)
    part = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0)
    return P, part, ie.Problem(2, n), dd.Partition(2, n, 16, 1, dd.CBD)


def _raw_factor(P, part, opts, ws_bytes, hint=None):
    """rs_factor_batched through ctypes with a workspace of exactly ws_bytes."""
    ws = torch.empty(max(ws_bytes, 256), dtype=torch.uint8, device=DEV)
    h, used = ctypes.c_void_p(), ctypes.c_size_t()
    cnt = ctypes.c_int()
    cbd.lib().rs_factor_rank_count(part.handle, ctypes.byref(opts), ctypes.byref(cnt))
    ranks = torch.zeros(max(cnt.value, 1), dtype=torch.int32, device=DEV)
    hp = None
    if hint is not None:
        hint = np.ascontiguousarray(hint, dtype=np.int32)
        hp = hint.ctypes.data_as(ctypes.c_void_p)
    rc = cbd.lib().rs_factor_batched(P.handle, part.handle, ctypes.byref(opts), hp,
                                     ctypes.c_void_p(ws.data_ptr()), ws_bytes, ctypes.c_void_p(ranks.data_ptr()),
                                     ctypes.byref(used), None, ctypes.byref(h))
    torch.cuda.synchronize()
    return rc, h, used.value, ranks, ws


def test_ranks_out_and_hinted_workspace(cfg):
    P, part, O, opart = cfg
    F1 = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    # ranks_out lists every compressed box in level and batch order
    want = []
    for l in range(F1.stats()["levels"]):
        want += F1.level(l)[0]
    assert F1.ranks.cpu().tolist()[:len(want)] == want and F1.n_ranks == len(want)
    # with the ranks as hints the workspace query is enough without a retry, and the
    # factor is the same (ranks schedule the QR only)
    F2 = cbd.Factor(P, part, tol=1e-8, n_pxy=64, rank_hint=F1.ranks.cpu())
    assert F2.ws_used <= F2.ws.numel()
    assert torch.equal(F1.ranks, F2.ranks)
    r = torch.tensor(synth.rhs(O.N, 3, seed=1), device=DEV)
    assert torch.equal(F1.apply(r), F2.apply(r))


def test_workspace_too_small_is_reported_and_exact_size_works(cfg):
    P, part, O, opart = cfg
    F1 = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    need = F1.ws_used
    opts = _lib.RSOpts(1e-8, 64, 1.5, cbd.PREC_FP64, 0, None, 0, 0, 0, 0, 64)
    # far too small: CBD_EWORKSPACE, and the reported bytes exceed what was given
    rc, h, used, _, _ = _raw_factor(P, part, opts, 1 << 16)
    assert rc == _lib.EWORKSPACE and used > (1 << 16)
    assert b"workspace too small" in cbd.lib().cbd_last_error()
    # the high-water mark of a successful run is enough to run again (rounded to 256 B)
    rc, h, used2, ranks, ws = _raw_factor(P, part, opts, (need + 255) // 256 * 256)
    assert rc == 0, cbd.lib().cbd_last_error()
    cbd.lib().rs_factor_free(h)
    assert torch.equal(ranks[:F1.n_ranks], F1.ranks[:F1.n_ranks])


def test_small_scratch_chunks_levels_with_the_same_result(cfg):
    # a workspace with little room beyond the factor storage splits every level into
    # chunks of boxes; the factor equals the unchunked one
    P, part, O, opart = cfg
    F1 = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    F2 = cbd.Factor(P, part, tol=1e-8, n_pxy=64, workspace_bytes=256 << 10)
    assert F2.schedule()["chunks"] > F1.schedule()["chunks"]
    r = torch.tensor(synth.rhs(O.N, 2, seed=2), device=DEV)
    assert rel(F2.apply(r).cpu().numpy(), F1.apply(r).cpu().numpy()) <= 1e-13


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_apply_in_column_blocks(cfg, prec):
    # apply buffers of 8 columns: 20 right-hand sides go through in blocks of 8, 8, 4
    P, part, O, opart = cfg
    F64 = cbd.Factor(P, part, tol=1e-8, n_pxy=64, precision=prec)
    F8 = cbd.Factor(P, part, tol=1e-8, n_pxy=64, precision=prec, apply_rhs=8)
    r = torch.tensor(synth.rhs(O.N, 20, seed=3), device=DEV)
    z64, z8 = F64.apply(r).cpu().numpy(), F8.apply(r).cpu().numpy()
    # blocks of 8 columns use the same per-box products as 16-column blocks
    for c in range(20):
        assert rel(z8[c], z64[c]) <= (1e-13 if prec == 0 else 1e-6)


def test_apply_sub_terms_sum_to_the_apply_and_match_the_oracle(cfg):
    P, part, O, opart = cfg
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    R = rs.RSPreconditioner(O, opart, 1e-8, n_pxy=64)
    r = synth.rhs(O.N, 2, seed=4)
    rt = torch.tensor(r, device=DEV)
    total = np.zeros_like(r)
    for i, sd in enumerate(opart.subdomains):
        zi = F.apply_sub(i, rt).cpu().numpy()
        outside = np.setdiff1d(np.arange(O.N), sd.index)
        assert np.all(zi[:, outside] == 0.0)
        ref = np.zeros_like(r)
        ref[:, sd.index] = R.apply_sub(i, r[:, sd.index].T).T
        assert rel(zi, ref) <= 1e-10
        total += zi
    assert rel(total, F.apply(rt).cpu().numpy()) <= 1e-14


@pytest.mark.parametrize("prec,tol,bound", [(0, 1e-8, 1e-5), (1, 1e-6, 1e-3)], ids=["fp64", "fp32"])
def test_subdomain_projection_fixes_vectors_on_its_support(cfg, prec, tol, bound):
    # l:subdomain: P_i = R_i^T A_i^{-1} R_i A, and P_i x = x for supp x in Omega_i.
    # With the RS factor in place of A_i^{-1} this holds to the factor's accuracy
    P, part, O, opart = cfg
    F = cbd.Factor(P, part, tol=tol, n_pxy=64, precision=prec)
    rng = np.random.default_rng(5)
    for i, sd in enumerate(opart.subdomains):
        x = np.zeros(O.N)
        x[sd.index] = rng.standard_normal(len(sd.index))
        xt = torch.tensor(x, device=DEV)
        px = F.apply_sub(i, P.matvec(xt)).cpu().numpy()
        err = rel(px, x)
        print("subdomain %d: |P_i x - x| / |x| = %.2e" % (i, err))
        assert err <= bound
        outside = np.setdiff1d(np.arange(O.N), sd.index)
        assert np.all(px[outside] == 0.0)


def test_apply_sub_rejects_bad_subdomain(cfg):
    P, part, O, opart = cfg
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    r = torch.zeros(1, O.N, dtype=torch.float64, device=DEV)
    with pytest.raises(cbd.CbdError):
        F.apply_sub(part.D, r)

"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded inputs.

Tolerances (FP64 path):
* matvec: 1e-13 relative to max|y| (summation order and one-ulp log/sqrt differences);
* ID coefficients T, E = B_sr G^{-1}, G^{-1}: 1e-7 relative (Frobenius).  A backward-stable
  T = R11^{-1} R12 has forward error ~ u * cond(R11) and cond(R11) <= 1/tol by the rank rule,
  so at tol = 1e-8 differences up to ~1e-8 are rounding, not error;
* B_ss, roots: 1e-8;  preconditioner apply: 1e-10;
* PCG: relative residual 1e-10 and solution within 1e-8 of the dense solve.
FP32 factors (ID still FP64): apply within 1e-4 of the FP64 oracle, PCG solution within 1e-8.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import cmatvec, dd, ie, pcg, precond, rs
from oracle.cpqr import interp_decomp

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2108_12574_amd as cbd

DEV = "cuda:0"


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def gpu_problem(d, n, coef=False):
    b = synth.coef_smooth(d, n) if coef else None
    bt = None if b is None else torch.tensor(b)
    P = cbd.Problem(d, n, b=bt, c=bt, device=DEV)
    O = ie.Problem(d, n, b=b, c=b)
    return P, O


@pytest.mark.parametrize("d,n,nrhs", [(2, 37, 1), (2, 37, 20), (2, 50, 64), (3, 11, 3), (3, 9, 17)])
def test_assemble_and_matvec(d, n, nrhs):
    print("case", d, n, nrhs, flush=True)
    P, O = gpu_problem(d, n, coef=True)
    assert np.array_equal(P.pts.cpu().numpy().reshape(d, -1).T, O.x)
    assert np.allclose(P.diag.cpu().numpy(), O.diag(), rtol=1e-15, atol=0)
    x = synth.rhs(O.N, nrhs, seed=1)
    y = P.matvec(torch.tensor(x, device=DEV)).cpu().numpy()
    yr = cmatvec.matvec(O, x.T).T
    assert np.abs(y - yr).max() <= 1e-13 * np.abs(yr).max()


@pytest.mark.parametrize("n,nrhs,coef", [(64, 1, True), (64, 20, False), (128, 5, True), (128, 64, True),
                                         (256, 3, False), (256, 70, True), (128, 1, False), (512, 1, True)])
def test_matvec_grid_table_form(n, nrhs, coef):
    # 2D grids whose lines hold whole workgroups (n a multiple of 64) take the entries
    # from per-tile tables of the grid offsets (one right-hand side: grid lines as the
    # MFMA columns); same product as the oracle's
    P, O = gpu_problem(2, n, coef=coef)
    x = synth.rhs(O.N, nrhs, seed=11)
    y = P.matvec(torch.tensor(x, device=DEV)).cpu().numpy()
    if n <= 128:
        ref = cmatvec.matvec(O, x.T).T
    else:
        rows = np.random.default_rng(3).choice(O.N, 64, replace=False)
        ref = cmatvec.matvec(O, x.T, rows=rows).T
        y = y[:, rows]
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("n", [24, 64])
def test_matvec_node_grid_and_single_rhs_vector(n):
    # n = 64 takes the table form with the node grid's spacing 1/(n - 1)
    P = cbd.Problem(2, n, grid=cbd.GRID_NODE, device=DEV)
    O = ie.Problem(2, n, grid=ie.GRID_NODE)
    x = synth.rhs(O.N, 1, seed=2)[0]
    y = P.matvec(torch.tensor(x, device=DEV)).cpu().numpy()
    assert y.shape == (O.N,)
    assert np.abs(y - O.dense() @ x).max() <= 1e-13 * np.abs(y).max()


def _compare_factor(F, R, opart, tol_T=1e-7):
    nbox = 0
    for i, sd in enumerate(opart.subdomains):
        for l in range(sd.root_level):
            for b in range(len(sd.levels[l])):
                g = F.box(i, l, b)
                o = R.subs[i].levels[l][b]
                assert np.array_equal(g["sk"], o.sk), (i, l, b)
                assert np.array_equal(g["rd"], o.rd), (i, l, b)
                if len(o.rd) and len(o.sk):
                    assert rel(g["T"], o.T) <= tol_T, (i, l, b, rel(g["T"], o.T))
                    assert rel(g["E"], o.E) <= tol_T, (i, l, b)
                if len(o.rd):
                    assert rel(g["Ginv"], np.linalg.inv(o.G)) <= tol_T, (i, l, b)
                if len(o.sk):
                    assert rel(g["Bss"], o.Bss) <= 1e-8, (i, l, b)
                nbox += 1
        idx, Gi = F.root(i)
        assert np.array_equal(idx, R.subs[i].root)
        assert rel(Gi, np.linalg.inv(R.subs[i].root_G)) <= 1e-8
    return nbox


CFG1 = dict(d=2, n=64, m=16, delta=1, mode=dd.CBD, leaf=0, tol=1e-8, npxy=64)


@pytest.fixture(scope="module")
def cfg1():
    P, O = gpu_problem(2, 64)
    part = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0)
    opart = dd.Partition(2, 64, 16, 1, dd.CBD)
    R = rs.RSPreconditioner(O, opart, 1e-8, n_pxy=64)
    return P, O, part, opart, R


def test_factor_fp64_matches_oracle_box_by_box(cfg1):
    P, O, part, opart, R = cfg1
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    assert _compare_factor(F, R, opart) == 4 * (64 + 16 + 4)
    st = F.stats()
    assert st["S"] == [len(s.root) for s in R.subs]
    assert st["levels"] == 3


def test_apply_fp64_matches_oracle(cfg1):
    P, O, part, opart, R = cfg1
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    r = synth.rhs(O.N, 20, seed=0)
    z = F.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    assert rel(z, R.apply(r.T).T) <= 1e-10
    # one column alone gives the same column
    z1 = F.apply(torch.tensor(r[3], device=DEV)).cpu().numpy()
    assert rel(z1, z[3]) <= 1e-14


def test_pcg_fp64_matches_dense_solve(cfg1):
    P, O, part, opart, R = cfg1
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    f = synth.rhs(O.N, 1, seed=0)[0]
    u, it, rr = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-10, maxit=200)
    A = O.dense()
    ud = np.linalg.solve(A, f)
    _, it_o, _ = pcg.pcg(lambda X: A @ X, R.apply, f, tol=1e-10, maxit=200)
    assert rr <= 1e-10
    assert abs(it - it_o) <= 1
    assert rel(u.cpu().numpy(), ud) <= 1e-8


def test_fp32_factor_and_pcg(cfg1):
    P, O, part, opart, R = cfg1
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64, precision=cbd.PREC_FP32)
    # the ID runs in FP64, so skeletons and ranks equal the FP64 oracle's
    for i, sd in enumerate(opart.subdomains):
        for b in range(len(sd.levels[0])):
            assert np.array_equal(F.box(i, 0, b)["sk"], R.subs[i].levels[0][b].sk)
    r = synth.rhs(O.N, 2, seed=0)
    z = F.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    assert rel(z, R.apply(r.T).T) <= 1e-4
    f = r[0]
    u, it, rr = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-10, maxit=200)
    ud = np.linalg.solve(O.dense(), f)
    assert rr <= 1e-10 and rel(u.cpu().numpy(), ud) <= 1e-8
    uf, itf, rrf = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-10, maxit=200, flexible=True)
    assert rrf <= 1e-10 and rel(uf.cpu().numpy(), ud) <= 1e-8


@pytest.mark.parametrize("mode,m,delta", [(2, 8, 1), (1, 2, 1), (0, 2, 0)],
                         ids=["cbd", "schwarz", "jacobi"])
def test_exact_subsolves_match_oracle(mode, m, delta):
    # naive preconditioners of Section 5.1 (table t:it_m48 settings) through the same kernels
    P, O = gpu_problem(2, 32)
    part = cbd.Partition(P, m, delta, mode, 0)
    F = cbd.Factor(P, part, exact=True)
    E = precond.ExactPreconditioner(O, dd.Partition(2, 32, m, delta, mode))
    r = synth.rhs(O.N, 3, seed=5)
    z = F.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    assert rel(z, E.apply(r.T).T) <= 1e-12
    f = synth.rhs(O.N, 1, seed=0)[0]
    u, it, rr = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-12, maxit=300)
    A = O.dense()
    _, it_o, _ = pcg.pcg(lambda X: A @ X, E.apply, f, tol=1e-12, maxit=300)
    assert abs(it - it_o) <= 1


@pytest.mark.parametrize("case", [
    dict(d=2, n=48, m=12, delta=1, mode=2, leaf=0, tol=1e-6, npxy=64, coef=True),     # variable coefficients
    dict(d=2, n=64, m=2, delta=8, mode=1, leaf=8, tol=1e-6, npxy=64, coef=False),     # Schwarz, leaf tiles
    dict(d=2, n=60, m=6, delta=2, mode=2, leaf=4, tol=1e-6, npxy=48, coef=False),     # CBD + tiles, ragged
    dict(d=3, n=16, m=4, delta=1, mode=2, leaf=0, tol=1e-6, npxy=256, coef=False),    # 3D
    dict(d=2, n=64, m=1, delta=0, mode=0, leaf=8, tol=1e-8, npxy=64, coef=False),     # global RS
    # sublinear partition counts (M ~ N^(6/7) in 2D, N^(3/4) in 3D, Section 4.4): partitions
    # of 3 x 3 and 2 x 2 x 2 points
    dict(d=2, n=120, m=40, delta=1, mode=2, leaf=0, tol=1e-6, npxy=64, coef=True),
    dict(d=3, n=12, m=6, delta=1, mode=2, leaf=0, tol=1e-6, npxy=256, coef=False),
], ids=["coef", "schwarz_tiles", "cbd_tiles", "3d", "global_rs", "sublinear_2d", "sublinear_3d"])
def test_factor_and_apply_other_layouts(case):
    print("case", case, flush=True)
    P, O = gpu_problem(case["d"], case["n"], case["coef"])
    part = cbd.Partition(P, case["m"], case["delta"], case["mode"], case["leaf"])
    opart = dd.Partition(case["d"], case["n"], case["m"], case["delta"], case["mode"], case["leaf"])
    R = rs.RSPreconditioner(O, opart, case["tol"], n_pxy=case["npxy"])
    F = cbd.Factor(P, part, tol=case["tol"], n_pxy=case["npxy"])
    _compare_factor(F, R, opart, tol_T=1e-8)
    r = synth.rhs(O.N, 4, seed=9)
    z = F.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    assert rel(z, R.apply(r.T).T) <= 1e-10


def test_multiple_rhs_and_edge_columns(cfg1):
    P, O, part, opart, R = cfg1
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    f = synth.rhs(O.N, 5, seed=3)
    f[2] = 0.0                       # a zero right-hand side converges at once
    U, its, rrs = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-10, maxit=200)
    U = U.cpu().numpy()
    assert its[2] == 0 and rrs[2] == 0.0 and np.all(U[2] == 0.0)
    for c in (0, 4):
        u1, it1, _ = cbd.pcg_solve(P, F, torch.tensor(f[c], device=DEV), tol=1e-10, maxit=200)
        assert it1 == its[c]
        assert rel(U[c], u1.cpu().numpy()) <= 1e-12


def test_not_converged_and_errors(cfg1):
    P, O, part, opart, R = cfg1
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    f = synth.rhs(O.N, 1, seed=0)[0]
    u, it, rr = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-10, maxit=1)
    assert it == 1 and rr > 1e-10
    # an indefinite operator (c = -b) is reported as not SPD, not factored
    b = torch.ones(O.N, dtype=torch.float64)
    Pn = cbd.Problem(2, 64, b=b, c=-b, device=DEV)
    with pytest.raises(cbd.CbdError) as e:
        cbd.Factor(Pn, part, tol=1e-8)
    assert e.value.code == -3 and "level 0" in str(e.value)
    with pytest.raises(cbd.CbdError):
        cbd.Factor(P, cbd.Partition((2, 32), 8), tol=1e-8)   # partition of another grid
    with pytest.raises(ValueError):
        P.matvec(torch.zeros(3, 10, dtype=torch.float64, device=DEV))


# ---- full-size workloads: sampled outputs and properties -----------------------

@pytest.fixture(scope="module")
def cfg3():
    n = 512
    P, O = gpu_problem(2, n, coef=True)
    part = cbd.Partition(P, 64, 1, cbd.MODE_CBD, 0)
    return P, O, part


def test_full_size_matvec_sampled_rows(cfg3):
    P, O, part = cfg3
    x = synth.rhs(O.N, 64, seed=0)
    y = P.matvec(torch.tensor(x, device=DEV)).cpu().numpy()
    rows = np.random.default_rng(0).choice(O.N, 24, replace=False)
    yr = cmatvec.matvec(O, x.T, rows=rows)          # (rows, 64)
    assert np.abs(y[:, rows].T - yr).max() <= 1e-12 * np.abs(yr).max()


@pytest.mark.parametrize("nrhs", [1, 64])
def test_full_size_1024_dense_matvec_sampled_rows(nrhs):
    # the dense product at 1024^2 (N = 1048576) with coefficients: one right-hand side
    # takes the grid-line form, 64 the table form; sampled rows against the oracle's C sum
    P, O = gpu_problem(2, 1024, coef=True)
    x = synth.rhs(O.N, nrhs, seed=2)
    y = P.matvec(torch.tensor(x, device=DEV)).cpu().numpy()
    rows = np.concatenate([[0, O.N - 1, 1023, O.N // 2], np.random.default_rng(3).choice(O.N, 12, replace=False)])
    yr = cmatvec.matvec(O, x.T, rows=rows)          # (rows, nrhs)
    assert np.abs(y[:, rows].T - yr).max() <= 1e-12 * np.abs(yr).max()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_full_size_leaf_ids_sampled(cfg3, prec):
    # the first level depends on geometry only: sampled leaf boxes' skeletons
    # equal the oracle's ID of the same box, computed one by one
    P, O, part = cfg3
    F = cbd.Factor(P, part, tol=1e-6, n_pxy=64, precision=prec)
    opart = dd.Partition(2, 512, 64, 1, dd.CBD)
    rng = np.random.default_rng(1)
    for i in range(4):
        sd = opart.subdomains[i]
        for b in rng.choice(len(sd.leaves), 3, replace=False):
            f1 = _single_leaf_factor(O, sd, b)
            g = F.box(i, 0, int(b))
            assert np.array_equal(g["sk"], f1[0]) and np.array_equal(g["rd"], f1[1])
            assert rel(g["T"], f1[2]) <= (1e-7 if prec == 0 else 1e-5)


def _single_leaf_factor(O, sd, b, tol=1e-6, npxy=64, ratio=1.5):
    lo, hi, st, cnt = sd.leaves[b]
    p = np.arange(st, st + cnt)
    others = np.setdiff1d(np.arange(len(sd.index)), p)
    lo, hi = np.array(lo), np.array(hi)
    J = np.stack([sd.index % O.n, sd.index // O.n], axis=1)
    off = 2 * J[others] + 1 - (lo + hi)
    near = others[np.sum(off * off, axis=1) < (2 * ratio * np.max(hi - lo)) ** 2]
    ctr = 0.5 * (lo + hi) / O.n
    rho = ratio * np.max(hi - lo) / O.n
    th = 2 * np.pi * np.arange(npxy) / npxy
    pxy = ctr + rho * np.stack([np.cos(th), np.sin(th)], axis=1)
    xp = O.x[sd.index[p]]
    Kp = -np.log(np.linalg.norm(pxy[:, None] - xp[None], axis=2)) / (2 * np.pi)
    Y = np.vstack([O.block(sd.index[near], sd.index[p]), Kp * O.weight * O.c[sd.index[p]]])
    k, perm, T = interp_decomp(Y, tol)
    return p[perm[:k]], p[perm[k:]], T


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_full_size_pcg_residual_sampled(cfg3, prec):
    # 512^2, 4 right-hand sides: recurrence residual <= 1e-10 and the true residual
    # f - A u, evaluated by the oracle on sampled rows, is of the same size
    P, O, part = cfg3
    F = cbd.Factor(P, part, tol=1e-6, n_pxy=64, precision=prec)
    f = synth.rhs(O.N, 4, seed=0)
    U, its, rrs = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-10, maxit=200)
    assert max(rrs) <= 1e-10 and max(its) <= 60
    U = U.cpu().numpy()
    rows = np.random.default_rng(2).choice(O.N, 64, replace=False)
    Au = cmatvec.matvec(O, U.T, rows=rows)          # (rows, 4)
    res = f[:, rows].T - Au
    # entries of f are O(1): sampled true residual RMS vs ||f||/sqrt(N)
    for c in range(4):
        rms = np.sqrt(np.mean(res[:, c] ** 2))
        assert rms <= 1e-8 * np.linalg.norm(f[c]) / np.sqrt(O.N)


@pytest.mark.parametrize("prec,flexible", [(0, False), (1, True)], ids=["fp64", "fp32_flexible"])
def test_pcg_graph_replay_matches_eager(cfg1, prec, flexible):
    # two captured graphs replayed every iteration, with host work and a
    # synchronization between replays; the result equals the eager solve bitwise
    P, O, part, opart, R = cfg1
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64, precision=prec)
    f = torch.tensor(synth.rhs(O.N, 3, seed=4), device=DEV)
    s = torch.cuda.Stream(device=DEV)
    with torch.cuda.stream(s):
        ue, ie_, re_ = cbd.pcg_solve(P, F, f, tol=1e-10, maxit=200, flexible=flexible)
        for rep in range(2):
            ug, ig, rg = cbd.pcg_solve(P, F, f, tol=1e-10, maxit=200, flexible=flexible, graph=True)
            s.synchronize()
            assert ig == ie_ and rg == re_
            assert torch.equal(ug, ue)
    assert max(re_) <= 1e-10


def test_autotune_matvec_keeps_results(cfg3):
    P, O, part = cfg3
    x = torch.tensor(synth.rhs(O.N, 64, seed=0), device=DEV)
    y0 = P.matvec(x)
    choice = P.autotune_matvec(64)
    assert choice in (1, 2, 4, 10, 12)
    y1 = P.matvec(x)
    assert torch.allclose(y0, y1, rtol=1e-13, atol=1e-13 * y0.abs().max().item())


@pytest.mark.parametrize("shape", [1, 2, 4, 9, 10, 12])
@pytest.mark.parametrize("nrhs", [20, 64])
def test_every_matvec_tile_shape_512(cfg3, shape, nrhs):
    # each tile shape of the table form (4 or 8 waves per workgroup, 1 to 4 row blocks
    # per wave) against the oracle on sampled rows
    P, O, part = cfg3
    x = synth.rhs(O.N, nrhs, seed=5)
    P.set_matvec_shape(nrhs, shape)
    try:
        y = P.matvec(torch.tensor(x, device=DEV)).cpu().numpy()
    finally:
        P.set_matvec_shape(nrhs, 4)
    rows = np.random.default_rng(shape).choice(O.N, 16, replace=False)
    ref = cmatvec.matvec(O, x.T, rows=rows).T
    assert np.abs(y[:, rows] - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_large_boxes_exact_subsolves(prec):
    # subdomains of 625 points: Cholesky and inverse by the multi-workgroup path
    # (blocked, batched over boxes), roots applied by GEMMs
    P, O = gpu_problem(2, 48)
    part = cbd.Partition(P, 2, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, exact=True, precision=prec)
    assert min(F.stats()["S"]) >= 512
    E = precond.ExactPreconditioner(O, dd.Partition(2, 48, 2, 1, dd.CBD))
    r = synth.rhs(O.N, 5, seed=6)
    z = F.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    assert rel(z, E.apply(r.T).T) <= (1e-11 if prec == 0 else 2e-4)


def test_large_roots_match_oracle():
    # 128^2, CBD m = 32, tol 1e-8: roots above 512 DOFs go through the multi-workgroup path
    P, O = gpu_problem(2, 128)
    part = cbd.Partition(P, 32, 1, cbd.MODE_CBD, 0)
    opart = dd.Partition(2, 128, 32, 1, dd.CBD)
    R = rs.RSPreconditioner(O, opart, 1e-8, n_pxy=64)
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    S = F.stats()["S"]
    print("roots", S, flush=True)
    assert min(S) >= 512
    for i in range(4):
        idx, Gi = F.root(i)
        assert np.array_equal(idx, R.subs[i].root)
        assert rel(Gi, np.linalg.inv(R.subs[i].root_G)) <= 1e-8
    r = synth.rhs(O.N, 3, seed=1)
    z = F.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    assert rel(z, R.apply(r.T).T) <= 1e-10


def test_bf16_gemm_variant(cfg1):
    # Schur-complement products on bfloat16 operands (FP32 accumulation): the
    # preconditioner is less accurate, FP64 PCG still reaches 1e-10 and the
    # solution still matches the dense solve
    P, O, part, opart, R = cfg1
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64, precision=cbd.PREC_BF16GEMM)
    r = synth.rhs(O.N, 2, seed=0)
    z = F.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    err = rel(z, R.apply(r.T).T)
    print("bf16 apply error vs FP64 oracle %.2e" % err, flush=True)
    assert err <= 5e-2
    f = r[0]
    u, it, rr = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-10, maxit=300, flexible=True)
    ud = np.linalg.solve(O.dense(), f)
    print("bf16 pcg iterations", it, flush=True)
    assert rr <= 1e-10 and rel(u.cpu().numpy(), ud) <= 1e-8


def _single_leaf_factor_3d(O, sd, b, tol=1e-6, npxy=256, ratio=1.5):
    lo, hi, st, cnt = sd.leaves[b]
    p = np.arange(st, st + cnt)
    others = np.setdiff1d(np.arange(len(sd.index)), p)
    lo, hi = np.array(lo), np.array(hi)
    n = O.n
    J = np.stack([sd.index % n, (sd.index // n) % n, sd.index // (n * n)], axis=1)
    off = 2 * J[others] + 1 - (lo + hi)
    near = others[np.sum(off * off, axis=1) < (2 * ratio * np.max(hi - lo)) ** 2]
    ctr = 0.5 * (lo + hi) / n
    R = ratio * np.max(hi - lo) / n
    pxy = ctr + R * rs.proxy_directions(3, npxy)
    xp = O.x[sd.index[p]]
    Kp = 1.0 / (4 * np.pi * np.linalg.norm(pxy[:, None] - xp[None], axis=2))
    Y = np.vstack([O.block(sd.index[near], sd.index[p]), Kp * O.weight * O.c[sd.index[p]]])
    k, perm, T = interp_decomp(Y, tol)
    return p[perm[:k]], T


def test_full_size_3d_sampled():
    # 3D 32^3, CBD m = 8, tol 1e-6, 256 proxy points, FP32 factors, 16 RHS:
    # sampled leaf IDs against the oracle, and the true residual on sampled rows
    P, O = gpu_problem(3, 32)
    part = cbd.Partition(P, 8, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-6, n_pxy=256, precision=cbd.PREC_FP32)
    opart = dd.Partition(3, 32, 8, 1, dd.CBD)
    rng = np.random.default_rng(3)
    for i in (0, 5):
        sd = opart.subdomains[i]
        for b in rng.choice(len(sd.leaves), 2, replace=False):
            sk, T = _single_leaf_factor_3d(O, sd, int(b))
            g = F.box(i, 0, int(b))
            assert np.array_equal(g["sk"], sk), (i, b)
            assert rel(g["T"], T) <= 1e-5
    f = synth.rhs(O.N, 16, seed=0)
    U, its, rrs = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-10, maxit=200)
    assert max(rrs) <= 1e-10 and max(its) <= 40
    rows = rng.choice(O.N, 48, replace=False)
    res = f[:, rows].T - cmatvec.matvec(O, U.cpu().numpy().T, rows=rows)
    for c in range(16):
        assert np.sqrt(np.mean(res[:, c] ** 2)) <= 1e-8 * np.linalg.norm(f[c]) / np.sqrt(O.N)


def test_full_size_schwarz_256_sampled_subdomains():
    # 256^2, Schwarz 4 x 4 subdomains, overlap one 8 x 8 leaf tile, tol 1e-6, FP64:
    # three of the sixteen subdomains (corner, edge, interior) compared box by box
    P, O = gpu_problem(2, 256)
    part = cbd.Partition(P, 4, 8, cbd.MODE_SCHWARZ, 8)
    F = cbd.Factor(P, part, tol=1e-6, n_pxy=64)
    opart = dd.Partition(2, 256, 4, 8, dd.SCHWARZ, 8)
    for i in (0, 1, 5):
        print("subdomain", i, flush=True)
        sd = opart.subdomains[i]
        f = rs.factor_subdomain(O, opart, sd, 1e-6, 64)
        for l in range(sd.root_level):
            for b in range(len(sd.levels[l])):
                g = F.box(i, l, b)
                o = f.levels[l][b]
                assert np.array_equal(g["sk"], o.sk) and np.array_equal(g["rd"], o.rd), (i, l, b)
                if len(o.rd) and len(o.sk):
                    assert rel(g["T"], o.T) <= 1e-8
        idx, Gi = F.root(i)
        assert np.array_equal(idx, f.root)
    fr = synth.rhs(O.N, 1, seed=0)[0]
    u, it, rr = cbd.pcg_solve(P, F, torch.tensor(fr, device=DEV), tol=1e-10, maxit=200)
    assert rr <= 1e-10 and it <= 40
    rows = np.random.default_rng(4).choice(O.N, 64, replace=False)
    res = fr[rows] - cmatvec.matvec(O, u.cpu().numpy(), rows=rows)
    assert np.sqrt(np.mean(res ** 2)) <= 1e-8 * np.linalg.norm(fr) / np.sqrt(O.N)


def test_full_size_1024_fft_sampled():
    # 1024^2, CBD m = 128, tol 1e-6, FP32 factors: sampled leaf IDs; PCG (FFT products)
    # to 1e-10 with the true residual checked by the oracle on sampled rows
    P, O = gpu_problem(2, 1024)
    part = cbd.Partition(P, 128, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-6, n_pxy=64, precision=cbd.PREC_FP32)
    opart = dd.Partition(2, 1024, 128, 1, dd.CBD)
    rng = np.random.default_rng(5)
    for i in (1, 2):
        sd = opart.subdomains[i]
        for b in rng.choice(len(sd.leaves), 2, replace=False):
            sk, rd, T = _single_leaf_factor(O, sd, int(b))
            g = F.box(i, 0, int(b))
            assert np.array_equal(g["sk"], sk)
    P.fft_prepare(max_pairs=1)
    fr = synth.rhs(O.N, 1, seed=0)[0]
    u, it, rr = cbd.pcg_solve(P, F, torch.tensor(fr, device=DEV), tol=1e-10, maxit=200, fft=True)
    assert rr <= 1e-10 and it <= 40
    rows = rng.choice(O.N, 16, replace=False)
    res = fr[rows] - cmatvec.matvec(O, u.cpu().numpy(), rows=rows)
    assert np.sqrt(np.mean(res ** 2)) <= 1e-8 * np.linalg.norm(fr) / np.sqrt(O.N)


@pytest.mark.parametrize("case", ["2d", "2d512", "3d"])
def test_row_compression_keeps_the_ids(case):
    # the pivoted QR on the Householder R of each tall proxy matrix picks the same
    # skeletons as on the matrix itself (equal column norms in exact arithmetic);
    # T agrees to the conditioning of R11.  2d512: the benchmark layout, whose
    # stepped levels have proxy matrices of up to about 2000 rows
    if case == "2d":
        P, _ = gpu_problem(2, 64)
        part, tol, npxy = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0), 1e-8, 64
    elif case == "2d512":
        P, _ = gpu_problem(2, 512, coef=True)
        part, tol, npxy = cbd.Partition(P, 64, 1, cbd.MODE_CBD, 0), 1e-6, 64
    else:
        P, _ = gpu_problem(3, 16)
        part, tol, npxy = cbd.Partition(P, 4, 1, cbd.MODE_CBD, 0), 1e-6, 256
    Fc = cbd.Factor(P, part, tol=tol, n_pxy=npxy, row_compression=cbd.ROWS_ALWAYS)
    Fp = cbd.Factor(P, part, tol=tol, n_pxy=npxy, row_compression=cbd.ROWS_NEVER)
    sc, sp = Fc.schedule(), Fp.schedule()
    print(case, "row-compressed levels", sc["row_compressed"], "vs", sp["row_compressed"], flush=True)
    assert sc["row_compressed"] > 0 and sp["row_compressed"] == 0
    nlev = Fc.stats()["levels"]
    for l in range(nlev):
        assert Fc.level(l) == Fp.level(l), l
    worst, nbox = 0.0, 0
    for l in range(nlev):
        count = {}
        subs = Fc.level(l)[2]
        if case == "2d512" and len(subs) >= 1024:
            continue   # levels of the one-workgroup QR: not row-compressed
        for i in subs:
            b = count.get(i, 0)
            count[i] = b + 1
            gc, gp = Fc.box(i, l, b), Fp.box(i, l, b)
            assert np.array_equal(gc["sk"], gp["sk"]) and np.array_equal(gc["rd"], gp["rd"]), (l, i, b)
            if gc["T"].size:
                worst = max(worst, rel(gc["T"], gp["T"]))
            nbox += 1
    print(case, nbox, "boxes, max rel T difference", worst, flush=True)
    assert worst <= 1e-6
    r = torch.tensor(synth.rhs(P.N, 2, seed=1), device=DEV)
    zc, zp = Fc.apply(r), Fp.apply(r)
    assert (zc - zp).norm() <= 1e-8 * zp.norm()


def test_global_rs_preconditioner_pcg():
    # global RS (one non-overlapping subdomain: the whole grid, 8 x 8 leaf tiles), the
    # paper's comparison system: at tol 1e-8 it is nearly the inverse, so PCG needs few
    # iterations; u against the oracle's dense solve
    P, O = gpu_problem(2, 64)
    part = cbd.Partition(P, 1, 0, cbd.MODE_JACOBI, 8)
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    assert len(F.stats()["S"]) == 1
    f = synth.rhs(O.N, 2, seed=0)
    u, it, rr = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-10, maxit=50)
    print("global RS: iterations", it, "root", F.stats()["S"], flush=True)
    assert max(it) <= 6 and max(rr) <= 1e-10
    ud = np.linalg.solve(O.dense(), f.T).T
    assert rel(u.cpu().numpy(), ud) <= 1e-8


@pytest.mark.parametrize("case", ["2d128", "64sq_tol1e-8", "3d16"])
def test_sketched_ids_match_oracle(case):
    # randomized IDs (random-sign sketch, same counter-based signs on both sides):
    # skeletons, T, E, G^{-1}, B_ss equal to the oracle's sketched RS box by box,
    # including the boxes whose sketch saturated and fell back
    if case == "2d128":
        d, n, m, tol, npxy = 2, 128, 16, 1e-6, 64
    elif case == "64sq_tol1e-8":
        d, n, m, tol, npxy = 2, 64, 16, 1e-8, 64
    else:
        d, n, m, tol, npxy = 3, 16, 4, 1e-4, 256     # the paper's 3D runs use loose tolerances
    P, O = gpu_problem(d, n)
    part = cbd.Partition(P, m, 1, cbd.MODE_CBD, 0)
    opart = dd.Partition(d, n, m, 1, dd.CBD)
    R = rs.RSPreconditioner(O, opart, tol, n_pxy=npxy, sketch_seed=12345)
    F = cbd.Factor(P, part, tol=tol, n_pxy=npxy, sketch_seed=12345)
    sch = F.schedule()
    osk = sum(s.sketched for s in R.subs)
    print(case, "sketched", sch["sketched"], "fallbacks", sch["sketch_fallbacks"], "oracle sketched", osk, flush=True)
    assert sch["sketched"] == osk and osk > 0
    nbox = _compare_factor(F, R, opart, tol_T=1e-7)
    assert sch["sketched"] <= nbox
    r = synth.rhs(O.N, 3, seed=4)
    z = F.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    assert rel(z, R.apply(r.T).T) <= 1e-10


def _hint_dict(opart, hint):
    """{(subdomain, level, box): rank} from a flat rank list in the factor's batch order
    (level by level; within a level subdomain by subdomain, boxes in partition order)."""
    out, h = {}, 0
    Lmax = max(sd.root_level for sd in opart.subdomains)
    for l in range(Lmax):
        for i, sd in enumerate(opart.subdomains):
            if sd.root_level <= l:
                continue
            for b in range(len(sd.levels[l])):
                out[(i, l, b)] = int(hint[h])
                h += 1
    assert h == len(hint)
    return out


@pytest.mark.parametrize("case,scale", [("2d64_m4", 1.0), ("2d64_m4", 0.5), ("3d32_m4", 1.0)])
def test_rank_sized_sketches_match_oracle(case, scale):
    # rank hints (a deterministic factorization's ranks, or half of them) size a first,
    # smaller sketch per box; kept when k <= rows / 4, else the shape-based sketch runs.
    # Box by box equal to the oracle's sketched RS given the same predictions
    if case == "2d64_m4":
        d, n, m, delta, mode, leaf, tol, npxy = 2, 64, 4, 1, dd.CBD, 0, 1e-6, 64
    else:    # the paper's 3D layout (8^3 points per partition) at its tolerance
        d, n, m, delta, mode, leaf, tol, npxy = 3, 32, 4, 1, dd.CBD, 0, 1e-3, 256
    P, O = gpu_problem(d, n)
    part = cbd.Partition(P, m, delta, mode, leaf)
    opart = dd.Partition(d, n, m, delta, mode, leaf)
    F0 = cbd.Factor(P, part, tol=tol, n_pxy=npxy)
    hint = (F0.ranks[:F0.n_ranks].cpu().numpy() * scale).astype(np.int32)
    F = cbd.Factor(P, part, tol=tol, n_pxy=npxy, sketch_seed=777, rank_hint=hint)
    R = rs.RSPreconditioner(O, opart, tol, n_pxy=npxy, sketch_seed=777, rank_pred=_hint_dict(opart, hint))
    sch = F.schedule()
    opred = sum(s.sketched_pred for s in R.subs)
    print(case, scale, "sketched", sch["sketched"], "rank-sized", sch["sketched_pred"], "rejected",
          sch["sketch_pred_rejected"], "oracle rank-sized", opred, flush=True)
    assert sch["sketched"] == sum(s.sketched for s in R.subs)
    assert sch["sketched_pred"] == opred
    if scale == 1.0:
        assert opred > 0
    else:
        assert sch["sketch_pred_rejected"] > 0
    _compare_factor(F, R, opart, tol_T=1e-7)
    r = synth.rhs(O.N, 3, seed=4)
    z = F.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    assert rel(z, R.apply(r.T).T) <= 1e-10


def test_sketched_ids_full_size_pcg():
    # 512^2 benchmark layout with randomized IDs (FP32 factors): PCG reaches 1e-10 in
    # about as many iterations as with deterministic IDs; true residual on sampled rows
    P, O = gpu_problem(2, 512, coef=True)
    part = cbd.Partition(P, 64, 1, cbd.MODE_CBD, 0)
    F0 = cbd.Factor(P, part, tol=1e-6, n_pxy=64, precision=cbd.PREC_FP32)
    F1 = cbd.Factor(P, part, tol=1e-6, n_pxy=64, precision=cbd.PREC_FP32, sketch_seed=1)
    sch = F1.schedule()
    print("sketched", sch["sketched"], "fallbacks", sch["sketch_fallbacks"], flush=True)
    assert sch["sketched"] > 0.9 * sum(len(F1.level(l)[0]) for l in range(F1.stats()["levels"]))
    f = synth.rhs(O.N, 2, seed=0)
    ft = torch.tensor(f, device=DEV)
    _, it0, _ = cbd.pcg_solve(P, F0, ft, tol=1e-10, maxit=200)
    u, it1, rr = cbd.pcg_solve(P, F1, ft, tol=1e-10, maxit=200)
    print("iterations deterministic", it0, "sketched", it1, flush=True)
    assert max(rr) <= 1e-10 and max(it1) <= max(it0) + 2
    rows = np.random.default_rng(2).choice(O.N, 32, replace=False)
    res = f[0][rows] - cmatvec.matvec(O, u[0].cpu().numpy(), rows=rows)
    assert np.sqrt(np.mean(res ** 2)) <= 1e-8 * np.linalg.norm(f[0]) / np.sqrt(O.N)


@pytest.mark.parametrize("case", ["cfg1", "cfg1_sketch", "big_roots"])
def test_chunked_levels_give_the_same_factors(case):
    # a small workspace budget splits every level into chunks of consecutive boxes;
    # each box's factor is the one of the unsplit level
    if case == "big_roots":
        P, _ = gpu_problem(2, 128)
        part, tol, seed = cbd.Partition(P, 8, 1, cbd.MODE_CBD, 0), 1e-6, None
    else:
        P, _ = gpu_problem(2, 64)
        part, tol = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0), 1e-8
        seed = 7 if case == "cfg1_sketch" else None
    # a generous workspace: no level is split
    big = torch.empty(1 << 30, dtype=torch.uint8, device=DEV)
    F0 = cbd.Factor(P, part, tol=tol, n_pxy=64, sketch_seed=seed, ws=big)
    F1 = cbd.Factor(P, part, tol=tol, n_pxy=64, sketch_seed=seed, workspace_bytes=2 << 20)
    s0, s1 = F0.schedule(), F1.schedule()
    nlev = F0.stats()["levels"]
    print(case, "chunks", s0["chunks"], "->", s1["chunks"], flush=True)
    assert s0["chunks"] == nlev + 1 and s1["chunks"] > s0["chunks"]
    for l in range(nlev + 1):
        assert F0.level(l) == F1.level(l), l
    for l in range(nlev):
        count = {}
        for i in F0.level(l)[2]:
            b = count.get(i, 0)
            count[i] = b + 1
            g0, g1 = F0.box(i, l, b), F1.box(i, l, b)
            assert np.array_equal(g0["sk"], g1["sk"]) and np.array_equal(g0["rd"], g1["rd"])
            # a chunk can send a batch to another form of the pivoted QR (register-resident
            # or streamed), whose sums run in another order: T, E, G^-1 agree to the
            # cond(R11)-limited tolerance of the oracle comparisons
            for key in ("T", "E", "Ginv", "Bss"):
                if g0[key].size:
                    assert rel(g1[key], g0[key]) <= 1e-7, (l, i, b, key)
    r = torch.tensor(synth.rhs(P.N, 2, seed=3), device=DEV)
    z0, z1 = F0.apply(r), F1.apply(r)
    assert (z1 - z0).norm() <= 1e-10 * z0.norm()


# Fixed N, varying partition count M (the paper's strong-scaling tables t:cbd_strong_2d and
# t:cbd_strong_3d: tolerance 1e-3, plain kernel without coefficients, proxy radius 1.5; the
# 3D rows there use randomized IDs).  S, the last-level size of a subdomain (the largest of
# the 4 or 8 here), grows as M^(1/2) in 2D and M^(2/3) in 3D (the paper's rank theorem), and
# the PCG iteration counts stay about constant.  Printed values from those tables: (m, S, n_it).
_STRONG = {
    "2d": dict(d=2, n=256, npxy=64, seed=None, rows=[(8, 64, 26), (16, 114, 26), (32, 213, 24), (64, 407, 22)]),
    "3d": dict(d=3, n=32, npxy=256, seed=1, rows=[(4, 527, 33), (8, 1358, 32), (16, 4120, 28)]),
}


@pytest.mark.parametrize("case", ["2d", "3d"])
def test_partition_count_sweep(case):
    import time
    c = _STRONG[case]
    d, n = c["d"], c["n"]
    P, O = gpu_problem(d, n)
    f = torch.tensor(synth.rhs(O.N, 1, seed=0)[0], device=DEV)
    S_prev = None
    for m, S_paper, it_paper in c["rows"]:
        part = cbd.Partition(P, m, 1, cbd.MODE_CBD, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = cbd.Factor(P, part, tol=1e-3, n_pxy=c["npxy"], proxy_ratio=1.5, sketch_seed=c["seed"])
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        S = max(F.stats()["S"])
        u, it, rr = cbd.pcg_solve(P, F, f, tol=1e-10, maxit=200)
        print("%s N=%d^%d M=%d^%d: S %d (paper %d), factor %.3f s, PCG iterations %d (paper %d), rel res %.2e"
              % (case, n, d, m, d, S, S_paper, tf, it, it_paper, rr), flush=True)
        assert rr <= 1e-10
        assert it <= it_paper + 10
        assert 0.5 * S_paper <= S <= 2.0 * S_paper
        if S_prev is not None:
            # 2^d times more partitions: S grows by about 2 (2D) or 4 (3D)
            lo, hi = (1.4, 2.6) if d == 2 else (2.0, 5.0)
            assert lo <= S / S_prev <= hi, (S_prev, S)
        S_prev = S


def test_sketched_leaf_ids_96cube_sampled():
    # 3D 96^3 (N/M = 512, 1728 leaf boxes of up to 1000 points), tol 1e-3, 256 proxy
    # points, randomized IDs, FP32 factors: the leaf level runs one workgroup per box on
    # sketches of up to 608 rows (the register-resident update up to 1024 rows); sampled
    # leaf IDs against the oracle's sketched ID of the same proxy matrix and signs
    from oracle import sketch
    P, O = gpu_problem(3, 96)
    part = cbd.Partition(P, 12, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-3, n_pxy=256, precision=cbd.PREC_FP32, sketch_seed=1)
    assert len(F.level(0)[0]) >= 1024
    opart = dd.Partition(3, 96, 12, 1, dd.CBD)
    rng = np.random.default_rng(6)
    n = O.n
    for i in (0, 7):
        sd = opart.subdomains[i]
        for b in rng.choice(len(sd.leaves), 2, replace=False):
            b = int(b)
            lo, hi, st, cnt = sd.leaves[b]
            p = np.arange(st, st + cnt)
            others = np.setdiff1d(np.arange(len(sd.index)), p)
            lo, hi = np.array(lo), np.array(hi)
            J = np.stack([sd.index % n, (sd.index // n) % n, sd.index // (n * n)], axis=1)
            off = 2 * J[others] + 1 - (lo + hi)
            near = others[np.sum(off * off, axis=1) < (2 * 1.5 * np.max(hi - lo)) ** 2]
            ctr = 0.5 * (lo + hi) / n
            pxy = ctr + 1.5 * np.max(hi - lo) / n * rs.proxy_directions(3, 256)
            xp = O.x[sd.index[p]]
            Kp = 1.0 / (4 * np.pi * np.linalg.norm(pxy[:, None] - xp[None], axis=2))
            Y = np.vstack([O.block(sd.index[near], sd.index[p]), Kp * O.weight * O.c[sd.index[p]]])
            rowkeys = np.concatenate([sd.index[near], O.N + np.arange(256)])
            k, perm, T, sketched = sketch.interp_decomp_sketched(Y, 1e-3, 1, sketch.box_key(i, 0, b), rowkeys)
            print("subdomain", i, "leaf", b, "Y", Y.shape, "k", k, "sketched", sketched, flush=True)
            assert sketched and sketch.sketch_size(*Y.shape) > 512
            g = F.box(i, 0, b)
            assert np.array_equal(g["sk"], p[perm[:k]]), (i, b)
            assert rel(g["T"], T) <= 1e-5


def test_leaf_ids_64cube_m16_sampled():
    # 3D 64^3, CBD m = 16 (4096 leaf boxes of up to 216 points), tol 1e-6, deterministic
    # IDs: the leaf level runs one workgroup per box on proxy matrices of 500 to 1300
    # rows (register-resident updates up to 1024 rows, two passes above); sampled leaf
    # IDs against the oracle
    P, O = gpu_problem(3, 64)
    part = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-6, n_pxy=256, precision=cbd.PREC_FP32)
    assert len(F.level(0)[0]) >= 1024
    X, _ = F.features(0)
    nnear = np.round(2.0 ** (8 * X[:, 3].astype(np.float64)) - 1)
    assert (nnear + 256 > 1024).any() and ((nnear + 256 > 512) & (nnear + 256 <= 1024)).any()
    opart = dd.Partition(3, 64, 16, 1, dd.CBD)
    rng = np.random.default_rng(8)
    for i in (2, 6):
        sd = opart.subdomains[i]
        for b in rng.choice(len(sd.leaves), 3, replace=False):
            sk, T = _single_leaf_factor_3d(O, sd, int(b))
            g = F.box(i, 0, int(b))
            assert np.array_equal(g["sk"], sk), (i, b)
            assert rel(g["T"], T) <= 1e-5


def test_leaf_ids_48cube_m4_sampled():
    # 3D 48^3, CBD m = 4 (64 leaf boxes of up to 2548 points), tol 1e-3, deterministic
    # IDs: the stepped QR runs on proxy matrices of about 2100 rows (the register-
    # resident update for 2048 to 3072 rows); sampled leaf IDs against the oracle
    P, O = gpu_problem(3, 48)
    part = cbd.Partition(P, 4, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-3, n_pxy=256, precision=cbd.PREC_FP32)
    opart = dd.Partition(3, 48, 4, 1, dd.CBD)
    rng = np.random.default_rng(9)
    for i in (1, 4):
        sd = opart.subdomains[i]
        for b in rng.choice(len(sd.leaves), 2, replace=False):
            sk, T = _single_leaf_factor_3d(O, sd, int(b), tol=1e-3)
            g = F.box(i, 0, int(b))
            assert np.array_equal(g["sk"], sk), (i, b)
            assert rel(g["T"], T) <= 1e-5


def test_global_rs_512_tall_levels():
    # 512^2 global RS (one subdomain, 8 x 8 leaf tiles), tol 1e-6: the top levels have
    # proxy matrices of more than 8192 rows, which must be row-compressed before the
    # stepped QR whatever the cost rule says; PCG on one right-hand side
    P, O = gpu_problem(2, 512, coef=True)
    part = cbd.Partition(P, 1, 0, cbd.MODE_JACOBI, 8)
    F = cbd.Factor(P, part, tol=1e-6, n_pxy=64, precision=cbd.PREC_FP32)
    sch = F.schedule()
    print("global 512^2: root", F.stats()["S"], "row-compressed levels", sch["row_compressed"], flush=True)
    assert sch["row_compressed"] >= 1
    f = torch.tensor(synth.rhs(O.N, 1, seed=0)[0], device=DEV)
    u, it, rr = cbd.pcg_solve(P, F, f, tol=1e-10, maxit=50)
    assert rr <= 1e-10 and it <= 6

"""GPU tests of the FFT matvec (circulant embedding; the paper's matvec on the uniform grid)."""
import numpy as np
import pytest
import torch

import synth
from oracle import cmatvec, dd, ie, rs

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2108_12574_amd as cbd

DEV = "cuda:0"


@pytest.mark.parametrize("d,n,nrhs,grid,coef", [(2, 37, 1, 0, True), (2, 37, 3, 0, True), (2, 64, 20, 0, False),
                                                (2, 24, 2, 1, False), (3, 11, 5, 0, True), (3, 16, 1, 0, False)])
def test_fft_matvec_matches_oracle(d, n, nrhs, grid, coef):
    print("case", d, n, nrhs, grid, coef, flush=True)
    b = synth.coef_smooth(d, n) if coef else None
    bt = None if b is None else torch.tensor(b)
    P = cbd.Problem(d, n, grid=grid, b=bt, c=bt, device=DEV)
    O = ie.Problem(d, n, grid=grid, b=b, c=b)
    P.fft_prepare(max_pairs=2)
    x = synth.rhs(O.N, nrhs, seed=1)
    y = P.matvec_fft(torch.tensor(x, device=DEV)).cpu().numpy()
    yr = cmatvec.matvec(O, x.T).T
    assert np.abs(y - yr).max() <= 1e-12 * np.abs(yr).max()


def test_fft_matvec_full_size_against_dense():
    n = 512
    b = torch.tensor(synth.coef_smooth(2, n))
    P = cbd.Problem(2, n, b=b, c=b, device=DEV)
    P.fft_prepare(max_pairs=8)
    x = torch.tensor(synth.rhs(n * n, 64, seed=0), device=DEV)
    y1 = P.matvec_fft(x)
    y0 = P.matvec(x)
    assert ((y1 - y0).abs().max() / y0.abs().max()).item() <= 1e-12


def test_pcg_with_fft_matvec():
    P = cbd.Problem(2, 64, device=DEV)
    O = ie.Problem(2, 64)
    part = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-8, n_pxy=64)
    P.fft_prepare()
    f = torch.tensor(synth.rhs(O.N, 3, seed=0), device=DEV)
    u0, i0, r0 = cbd.pcg_solve(P, F, f, tol=1e-10, maxit=200)
    u1, i1, r1 = cbd.pcg_solve(P, F, f, tol=1e-10, maxit=200, fft=True)
    assert max(r1) <= 1e-10
    assert all(abs(a - b) <= 1 for a, b in zip(i0, i1))
    ud = np.linalg.solve(O.dense(), f.cpu().numpy().T).T
    assert np.linalg.norm(u1.cpu().numpy() - ud) <= 1e-8 * np.linalg.norm(ud)
    with pytest.raises(cbd.CbdError):
        Q = cbd.Problem(2, 32, device=DEV)
        cbd.pcg_solve(Q, None, torch.zeros(Q.N, dtype=torch.float64, device=DEV), fft=True)

"""GPU tests of the IDs from the pivoted Cholesky of the Gram matrix (CBD_ID_GRAM).

In exact arithmetic these IDs are the truncated column-pivoted QR's of (e:id)
(tests/test_gram_reading.py checks that on the CPU); in FP64 rounding can move a
pivot at a near tie or the stopping step by one, so the skeletons are not compared
with the oracle's one by one.  What is unique is checked instead:
* the ID's own bound: every residual column Y_r - Y_s T of every box, rebuilt in
  FP64 by the oracle (oracle.rs.proxy_matrix) from the GPU's own active DOFs, within
  2 tol nu_0 (the QR's stopping rule gives tol nu_0; the QR form is held to 1.5);
* the preconditioner against the oracle's (QR IDs) on the same inputs, the PCG
  iteration count, and the solution against a dense solve.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import dd, ie, pcg, rs

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2108_12574_amd as cbd

DEV = "cuda:0"


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _id_bound(F, O, opart, tol, npxy):
    """Largest max_c |Y_r[:, c] - Y_s T[:, c]| / (tol nu_0) over the boxes (at most about
    64 per subdomain and level, evenly spaced), Y rebuilt by the oracle for the GPU's
    active DOFs."""
    worst, nbox = 0.0, 0
    for i, sd in enumerate(opart.subdomains):
        for l in range(sd.root_level):
            boxes = [F.box(i, l, b) for b in range(len(sd.levels[l]))]
            act = [np.concatenate([g["sk"], g["rd"]]).astype(np.int64) for g in boxes]
            allact = np.concatenate(act)
            step = max(1, len(boxes) // 64)
            for b, g in enumerate(boxes):
                if b % step:
                    continue
                k, nr = len(g["sk"]), len(g["rd"])
                if k == 0 or nr == 0:
                    continue
                Y, _ = rs.proxy_matrix(O, sd, sd.levels[l][b], act[b], np.setdiff1d(allact, act[b]), npxy)
                nu0 = np.linalg.norm(Y, axis=0).max()
                res = Y[:, k:] - Y[:, :k] @ g["T"]
                worst = max(worst, np.linalg.norm(res, axis=0).max() / (tol * nu0))
                nbox += 1
    return worst, nbox


def _agreement(Fa, Fb, nlev):
    same = total = 0
    for l in range(nlev):
        ka, _, subs = Fa.level(l)
        kb = Fb.level(l)[0]
        total += len(ka)
        same += sum(int(x == y) for x, y in zip(ka, kb))
    return same / max(total, 1)


CASES = {
    # name: (d, n, m, coefficients, tol, n_pxy)
    "2d64": (2, 64, 16, False, 1e-6, 64),
    "2d512": (2, 512, 64, True, 1e-6, 64),
    "3d16": (3, 16, 4, False, 1e-6, 256),
    "3d32": (3, 32, 8, False, 1e-6, 256),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_gram_ids_meet_the_qr_stopping_bound(case):
    d, n, m, coef, tol, npxy = CASES[case]
    b = synth.coef_smooth(d, n) if coef else None
    bt = None if b is None else torch.tensor(b)
    P = cbd.Problem(d, n, b=bt, c=bt, device=DEV)
    O = ie.Problem(d, n, b=b, c=b)
    part = cbd.Partition(P, m, 1, cbd.MODE_CBD, 0)
    opart = dd.Partition(d, n, m, 1, dd.CBD)
    Fq = cbd.Factor(P, part, tol=tol, n_pxy=npxy, id_method=cbd.ID_QR)
    Fg = cbd.Factor(P, part, tol=tol, n_pxy=npxy, id_method=cbd.ID_GRAM)
    wq, nq = _id_bound(Fq, O, opart, tol, npxy)
    wg, ng = _id_bound(Fg, O, opart, tol, npxy)
    agree = _agreement(Fq, Fg, Fq.stats()["levels"])
    print("%s: residual / (tol nu0): QR %.3f (%d boxes), Gram %.3f (%d boxes); equal ranks %.3f; "
          "panel launch pairs %d vs stepped %d" % (case, wq, nq, wg, ng, agree, Fg.schedule()["qr_steps"],
                                                   Fq.schedule()["qr_steps"]), flush=True)
    assert nq > 0 and ng > 0
    assert wq <= 1.5 and wg <= 2.0
    assert agree >= 0.8
    # the two factors are preconditioners of the same quality
    r = torch.tensor(synth.rhs(P.N, 2, seed=3), device=DEV)
    zq, zg = Fq.apply(r), Fg.apply(r)
    assert (zq - zg).norm() <= 1e-3 * zq.norm()


def test_gram_factor_apply_and_pcg_against_oracle():
    P = cbd.Problem(2, 64, device=DEV)
    O = ie.Problem(2, 64)
    part = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0)
    opart = dd.Partition(2, 64, 16, 1, dd.CBD)
    R = rs.RSPreconditioner(O, opart, 1e-6, n_pxy=64)
    Fg = cbd.Factor(P, part, tol=1e-6, n_pxy=64, id_method=cbd.ID_GRAM)
    r = synth.rhs(O.N, 4, seed=5)
    zg = Fg.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    err = rel(zg, R.apply(r.T).T)
    f = synth.rhs(O.N, 1, seed=6)[0]
    u, it, rr = cbd.pcg_solve(P, Fg, torch.tensor(f, device=DEV), tol=1e-10, maxit=200)
    A = O.dense()
    _, it_o, _ = pcg.pcg(lambda X: A @ X, R.apply, f, tol=1e-10, maxit=200)
    u_d = np.linalg.solve(A, f)
    print("apply vs oracle %.2e; iterations %d (oracle %d); u vs dense %.2e"
          % (err, it, it_o, rel(u.cpu().numpy(), u_d)), flush=True)
    assert err <= 1e-4
    assert abs(it - it_o) <= 1 and rr <= 1e-10
    assert rel(u.cpu().numpy(), u_d) <= 1e-8


def test_gram_needs_a_tolerance_above_its_rounding_floor():
    P = cbd.Problem(2, 64, device=DEV)
    part = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0)
    with pytest.raises(cbd.CbdError) as e:
        cbd.Factor(P, part, tol=1e-8, n_pxy=64, id_method=cbd.ID_GRAM)
    assert e.value.code == -1


def test_gram_route_with_sketches_chunks_and_hints():
    # the Gram route composes with the other factorization options: random-sign sketches
    # (the ID of Z = Omega Y), levels split into chunks by a small workspace, and rank
    # hints; the chunked and hinted factors equal the plain one
    P = cbd.Problem(3, 16, device=DEV)
    O = ie.Problem(3, 16)
    part = cbd.Partition(P, 4, 1, cbd.MODE_CBD, 0)
    opart = dd.Partition(3, 16, 4, 1, dd.CBD)
    kw = dict(tol=1e-3, n_pxy=256, sketch_seed=1, id_method=cbd.ID_GRAM)
    F = cbd.Factor(P, part, **kw)
    sc = F.schedule()
    assert sc["sketched"] > 0
    # a sketched ID meets the tolerance on Z = Omega Y; on Y its residual is held to the
    # bound the oracle's sketched pins use (30 tol nu_0), beside the QR route's
    w, nb = _id_bound(F, O, opart, 1e-3, 256)
    wq, _ = _id_bound(cbd.Factor(P, part, tol=1e-3, n_pxy=256, sketch_seed=1, id_method=cbd.ID_QR), O, opart,
                      1e-3, 256)
    print("sketched IDs: residual / (tol nu0) Gram %.3f, QR %.3f over %d boxes, %d sketched"
          % (w, wq, nb, sc["sketched"]), flush=True)
    assert w <= 30.0
    Fc = cbd.Factor(P, part, workspace_bytes=16 << 20, **kw)
    Fh = cbd.Factor(P, part, rank_hint=F.ranks.cpu(), **kw)
    assert Fc.schedule()["chunks"] > sc["chunks"]
    r = torch.tensor(synth.rhs(P.N, 2, seed=7), device=DEV)
    z = F.apply(r)
    for G in (Fc, Fh):
        assert torch.equal(G.ranks, F.ranks)
        assert (G.apply(r) - z).norm() <= 1e-12 * z.norm()


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "fp32"])
def test_gram_route_pcg_against_dense_solve(prec):
    P = cbd.Problem(2, 64, device=DEV)
    O = ie.Problem(2, 64)
    part = cbd.Partition(P, 8, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-6, n_pxy=64, precision=prec, id_method=cbd.ID_GRAM)
    f = synth.rhs(O.N, 1, seed=8)[0]
    u, it, rr = cbd.pcg_solve(P, F, torch.tensor(f, device=DEV), tol=1e-10, maxit=200)
    ud = np.linalg.solve(O.dense(), f)
    print("Gram route %s: %d iterations, u vs dense %.2e" % (("fp64", "fp32")[prec], it, rel(u.cpu().numpy(), ud)))
    assert rr <= 1e-10 and rel(u.cpu().numpy(), ud) <= 1e-8

"""GPU tests of the factorization's graph replay (rs_factor_capture, rs_factor_replay).

A replay re-runs every kernel of the factorization (Section 4.2) on the problem's
current device data and checks each value the eager run read back (ranks, skeleton
lists, stop flags, predictions, breakdown slots) against the recording.  Checked here:
* on unchanged data every replay reproduces the eager factor bit for bit (the apply of
  64 columns compared with torch.equal), three replays in a row with eager work of the
  program (another factorization, a PCG solve, synchronizations) between them; for
  both ID routes, both storage precisions, and with sketches, a rank predictor, rank
  hints, row compression and levels processed in chunks (every kind of upload and read
  the factorization makes);
* with different coefficients written into the problem's arrays the replay reports that
  its reads differ (CBD_EREPLAN), the factor is refused afterwards, and an eager
  factorization of the new data is unaffected;
* capture and replay refuse a factor made without a recording, and a replay before a
  capture.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2108_12574_amd as cbd

DEV = "cuda:0"


def _problem(n=128, coef=None):
    c = torch.tensor(synth.coef_smooth(2, n) if coef is None else coef)
    return cbd.Problem(2, n, b=c, c=c, device=DEV)


FORMS = {
    "qr_fp32": dict(precision=1, id_method=0),
    "gram_fp64": dict(precision=0, id_method=1),
    "qr_sketch_mlp_chunked_rows": dict(precision=1, id_method=0, sketch_seed=7, workspace_bytes=3 << 20,
                                       row_compression=2, mlp="init"),
    "gram_fp32_hint": dict(precision=1, id_method=1, hint=True),
}


def _opts(P, part, form):
    kw = dict(FORMS[form])
    if kw.pop("mlp", None):
        kw["mlp"] = cbd.RankMLP(omlp.init_params(3), DEV)
    if kw.pop("hint", False):
        kw["rank_hint"] = cbd.Factor(P, part, tol=1e-6, precision=kw["precision"], id_method=kw["id_method"]).ranks
    return kw


@pytest.mark.parametrize("form", list(FORMS))
def test_replay_reproduces_eager_factor(form):
    P = _problem()
    part = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0)
    kw = _opts(P, part, form)
    F = cbd.Factor(P, part, tol=1e-6, record=True, **kw)
    sched = F.schedule()
    if form.startswith("qr_sketch"):
        assert sched["chunks"] > F.stats()["levels"] + 1, sched   # some level ran in chunks
        assert sched["sketched"] > 0 and sched["row_compressed"] > 0, sched
    gen = torch.Generator(device=DEV).manual_seed(0)
    R = torch.randn(64, P.N, dtype=torch.float64, device=DEV, generator=gen)
    z0 = F.apply(R)
    ranks0 = F.ranks.clone()
    F.capture()
    f = torch.tensor(synth.rhs(P.N, 1, seed=1)[0], device=DEV)
    for rep in range(3):
        # eager work of the program between replays: a second factorization and a solve
        E = cbd.Factor(P, part, tol=1e-6, **kw)
        zE = E.apply(R)
        u, it, rr = cbd.pcg_solve(P, E, f, tol=1e-10, maxit=200)
        torch.cuda.synchronize()
        del E
        assert F.replay(), "replay %d did not reproduce the recording" % rep
        z = F.apply(R)
        print("%s replay %d: max |z - z_eager| = %.3e, eager factor again: %.3e, pcg %d its"
              % (form, rep, (z - z0).abs().max().item(), (zE - z0).abs().max().item(), it))
        assert torch.equal(z, z0)
        assert torch.equal(zE, z0)
        assert rr <= 1e-10
    assert torch.equal(F.ranks, ranks0)   # the replay writes no ranks_out
    assert F.schedule() == sched          # host-side statistics are the eager run's


def test_replay_detects_changed_ranks():
    P = _problem()
    part = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-6, precision=1, record=True)
    F.capture()
    assert F.replay()
    # coefficients with much more variation: the eager ranks differ
    x = (np.arange(128) + 0.5) / 128
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    coef2 = (1.0 + 0.9 * np.sin(6 * np.pi * X1) * np.cos(4 * np.pi * X2)).reshape(-1, order="F")
    P2 = _problem(coef=coef2)
    F2 = cbd.Factor(P2, part, tol=1e-6, precision=1)
    assert not torch.equal(F2.ranks, F.ranks)
    for name in ("pts", "diag", "w", "rowscale"):
        getattr(P, name).copy_(getattr(P2, name))
    torch.cuda.synchronize()
    assert not F.replay()
    R = torch.randn(4, P.N, dtype=torch.float64, device=DEV)
    with pytest.raises(cbd.CbdError) as e:
        F.apply(R)
    assert e.value.code == cbd._lib.EREPLAN
    assert not F.replay()   # a stale factor stays refused
    # a fresh eager factorization of the new data in P equals the one of P2
    F3 = cbd.Factor(P, part, tol=1e-6, precision=1)
    assert torch.equal(F3.ranks, F2.ranks)
    assert torch.equal(F3.apply(R), F2.apply(R))


def test_capture_and_replay_refuse_misuse():
    P = _problem(64)
    part = cbd.Partition(P, 8, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-6, precision=1)
    with pytest.raises(ValueError):
        F.capture()
    with pytest.raises(cbd.CbdError):
        F.replay()
    G = cbd.Factor(P, part, tol=1e-6, precision=1, record=True)
    with pytest.raises(cbd.CbdError):
        G.replay()

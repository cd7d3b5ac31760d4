"""GPU tests of the apply's per-level tile choice (cbd_autotune_apply, cbd_apply_set_shape).

The columns one workgroup of a level sweep takes, and its waves, change only how the
right-hand sides and the product tiles are spread: from 8 columns on every column's
sums run on matrix cores in the same order, so T^{-1} r ((e:ad)) must come out bit for
bit the same for every choice.  The
oracle comparison of the apply itself is in test_gpu_parity.py; here the tuned and
fixed shapes are held to the default shape's result, and invalid shapes are refused.
"""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2108_12574_amd as cbd

DEV = "cuda:0"


@pytest.mark.parametrize("prec,n,nrhs", [(1, 128, 64), (0, 128, 64), (1, 64, 4)])
def test_tuned_and_fixed_shapes_give_the_default_result(prec, n, nrhs):
    coef = torch.tensor(synth.coef_smooth(2, n))
    P = cbd.Problem(2, n, b=coef, c=coef, device=DEV)
    part = cbd.Partition(P, 16, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-6, precision=prec)
    R = torch.tensor(synth.rhs(P.N, nrhs, seed=2), device=DEV)
    z0 = F.apply(R)
    choices = F.autotune_apply(R)
    nlev = F.stats()["levels"] + 1
    assert len(choices) == nlev
    assert all(c in (0, 8, 16, 32, 64) and t in (0, 256, 512, 1024) for c, t in choices), choices
    print("prec %d n %d nrhs %d: columns per level %s" % (prec, n, nrhs, choices))
    assert torch.equal(F.apply(R), z0)
    for cols in (8, 16, 32, 64):
        for threads in (256, 512, 1024):
            try:
                F.set_apply_shapes([(cols, threads)] * nlev)
            except cbd.CbdError:
                continue   # some level's boxes need more LDS at this width
            assert torch.equal(F.apply(R), z0), (cols, threads)
    F.set_apply_shapes([(0, 0)] * nlev)
    assert torch.equal(F.apply(R), z0)


def test_bad_shapes_are_refused():
    P = cbd.Problem(2, 64, device=DEV)
    part = cbd.Partition(P, 8, 1, cbd.MODE_CBD, 0)
    F = cbd.Factor(P, part, tol=1e-6, precision=1)
    with pytest.raises(cbd.CbdError):
        F.set_apply_shapes([(12, 256)])
    with pytest.raises(cbd.CbdError):
        F.set_apply_shapes([(16, 768)])
    with pytest.raises(cbd.CbdError):
        F.set_apply_shapes([(16, 256)] * (F.stats()["levels"] + 2))   # one level too many

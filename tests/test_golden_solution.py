"""The stored oracle solutions (tests/golden/u_*_cbd_col0.npy) against their definition.

Each was written by tests/golden/make_solution_fixture.py from the oracle's RS-PCG
to relative residual 1e-12.  Here u is checked against what fixes it whatever
solver produced it: the true residual ||f - A u|| / ||f|| of A u = f (Section 2.1),
with A applied by the oracle's FFT product (itself pinned against the dense sum).
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import fftmv, ie

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("name", ["u_128sq_cbd_col0", "u_512sq_cbd_col0"])
def test_stored_solution_solves_the_system(name):
    rec = json.load(open(os.path.join(GOLD, name + ".json")))
    u = np.load(os.path.join(GOLD, name + ".npy"))
    d, n = rec["d"], rec["n"]
    N = n ** d
    assert u.shape == (N,) and u.dtype == np.float64
    coef = synth.coef_smooth(d, n)
    prob = ie.Problem(d, n, b=coef, c=coef)
    f = synth.rhs(N, 1, seed=0)[0]
    res = np.linalg.norm(f - fftmv.FFTMatvec(prob)(u)) / np.linalg.norm(f)
    assert res <= 1e-12, res
    assert np.linalg.norm(u) == pytest.approx(rec["u_norm"], rel=1e-14)

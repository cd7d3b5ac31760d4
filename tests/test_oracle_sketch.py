"""Pins of the sketched (randomized) ID of the oracle: the random-sign generator
against its published definition, exactness on matrices of known rank, the
fallback rule, and the ID error on real proxy matrices."""
import numpy as np
import pytest

from oracle import cpqr, dd, ie, rs, sketch


def test_splitmix64_output_function():
    # splitmix64 from state 0: the first output is mix64(0x9E3779B97F4A7C15)
    # = 0xE220A8397B1DCDAF (the generator's published first value)
    v = sketch.mix64(np.array([0x9E3779B97F4A7C15], dtype=np.uint64))
    assert int(v[0]) == 0xE220A8397B1DCDAF


def test_signs_are_balanced_and_uncorrelated():
    om = sketch.signs(7, sketch.box_key(1, 2, 3), 200, np.arange(1000))
    assert set(np.unique(om)) == {-1.0, 1.0}
    assert abs(om.mean()) < 0.01
    c = om @ om.T / om.shape[1]
    off = c[~np.eye(200, dtype=bool)]
    assert np.abs(off).max() < 0.2 and abs(off.mean()) < 0.01
    # a different box key or seed gives different signs
    assert not np.array_equal(om, sketch.signs(7, sketch.box_key(1, 2, 4), 200, np.arange(1000)))
    assert not np.array_equal(om, sketch.signs(8, sketch.box_key(1, 2, 3), 200, np.arange(1000)))


def test_sketch_size_rule():
    assert sketch.sketch_size(400, 100) == 68          # ceil(300/5) + 8
    assert sketch.sketch_size(60, 100) == 0             # not below min(m, n)
    assert sketch.sketch_size(1000, 7) == 0


@pytest.mark.parametrize("r", [5, 20, 40])
def test_exact_low_rank_is_reproduced(r):
    # Y = U V of rank r: the sketch has the same column dependencies, so its ID is exact
    rng = np.random.default_rng(r)
    m, n = 300, 90
    Y = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    k, perm, T, used = sketch.interp_decomp_sketched(Y, 1e-12, 3, 11, np.arange(m))
    assert used and k == r
    err = np.linalg.norm(Y[:, perm[k:]] - Y[:, perm[:k]] @ T)
    assert err <= 1e-10 * np.linalg.norm(Y)


def test_saturated_sketch_falls_back_to_the_deterministic_id():
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((300, 90))                  # full rank 90 > ell - 8 = 54
    k, perm, T, used = sketch.interp_decomp_sketched(Y, 1e-12, 3, 11, np.arange(300))
    k2, perm2, T2 = cpqr.interp_decomp(Y, 1e-12)
    assert not used and k == k2 and np.array_equal(perm, perm2) and np.array_equal(T, T2)


def test_sketched_rs_id_error_on_proxy_matrices():
    # every sketched ID of a 32^2 RS factorization meets the accuracy target against
    # the full far field of its box (all other points of the subdomain), as the
    # deterministic ID does, up to a modest factor
    O = ie.Problem(2, 32)
    part = dd.Partition(2, 32, 4, 1, dd.CBD)
    tol = 1e-6
    sd = part.subdomains[0]
    f = rs.factor_subdomain(O, part, sd, tol, 64, sketch_seed=5, sub=0)
    assert f.sketched > 0
    g = sd.index
    worst = 0.0
    for b in f.levels[0]:
        p = np.concatenate([b.sk, b.rd])
        far = np.setdiff1d(np.arange(len(g)), p)
        Y = O.block(g[far], g[p])
        Ysk, Yrd = O.block(g[far], g[b.sk]), O.block(g[far], g[b.rd])
        if len(b.rd):
            worst = max(worst, np.linalg.norm(Yrd - Ysk @ b.T) / np.linalg.norm(Y))
    print("worst relative far-field ID error", worst)
    assert worst <= 30 * tol


def test_sketched_preconditioner_keeps_the_iteration_count():
    # 128^2, CBD m = 16, tol 1e-6: every ID is sketched; PCG needs as many iterations
    # as with the deterministic IDs (the paper's randomized runs keep n_it)
    from oracle import pcg
    import synth
    O = ie.Problem(2, 128)
    part = dd.Partition(2, 128, 16, 1, dd.CBD)
    R0 = rs.RSPreconditioner(O, part, 1e-6, n_pxy=64)
    R1 = rs.RSPreconditioner(O, part, 1e-6, n_pxy=64, sketch_seed=1)
    nb = sum(len(l) for s in R1.subs for l in s.levels)
    assert sum(s.sketched for s in R1.subs) == nb
    f = synth.rhs(O.N, 1, seed=0)[0]
    A = O.dense()
    it0 = pcg.pcg(lambda x: A @ x, R0.apply, f, tol=1e-10, maxit=200)[1]
    it1 = pcg.pcg(lambda x: A @ x, R1.apply, f, tol=1e-10, maxit=200)[1]
    assert abs(it1 - it0) <= 1


def test_predicted_sketch_size_rule():
    # 4 k_p + 32 rows when below the shape-based size, else none
    assert sketch.predicted_sketch_size(400, 300, 10) == 72        # shape size 188
    assert sketch.predicted_sketch_size(400, 300, 38) == 184
    assert sketch.predicted_sketch_size(400, 300, 40) == 0         # 192 >= 188
    assert sketch.predicted_sketch_size(60, 300, 1) == 0           # no sketch at all


@pytest.mark.parametrize("r", [5, 20, 35])
def test_predicted_size_sketch_is_exact_on_low_rank(r):
    rng = np.random.default_rng(r)
    m, n = 400, 300
    Y = rng.standard_normal((m, r)) @ rng.standard_normal((r, n))
    k, perm, T, used = sketch.interp_decomp_sketched(Y, 1e-12, 3, 11, np.arange(m), k_pred=r)
    assert used and k == r
    assert np.linalg.norm(Y[:, perm[k:]] - Y[:, perm[:k]] @ T) <= 1e-10 * np.linalg.norm(Y)


def test_rejected_prediction_gives_the_shape_sketch():
    # rank 20 with a prediction of 0: the 32-row sketch finds k = 20 > 32/4, so the box
    # goes on to the shape-based sketch, and the result is the one without a prediction
    rng = np.random.default_rng(1)
    m, n = 400, 300
    Y = rng.standard_normal((m, 20)) @ rng.standard_normal((20, n))
    a = sketch.interp_decomp_sketched(Y, 1e-12, 3, 11, np.arange(m), k_pred=0)
    b = sketch.interp_decomp_sketched(Y, 1e-12, 3, 11, np.arange(m))
    assert a[0] == b[0] == 20 and a[3] and b[3]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


@pytest.mark.parametrize("scale", [1.0, 0.5])
def test_predicted_size_sketched_rs_id_error(scale):
    # 64^2 with 4^2 partitions (boxes of 324 points), tol 1e-6: with predictions equal to
    # (or half) the deterministic ranks, every ID still meets the accuracy target against
    # the box's full far field
    O = ie.Problem(2, 64)
    part = dd.Partition(2, 64, 4, 1, dd.CBD)
    tol = 1e-6
    sd = part.subdomains[0]
    f0 = rs.factor_subdomain(O, part, sd, tol, 64)
    pred = {(0, b): int(scale * len(bf.sk)) for b, bf in enumerate(f0.levels[0])}
    assert all(sketch.predicted_sketch_size(400, len(bf.sk) + len(bf.rd), pred[(0, b)])
               for b, bf in enumerate(f0.levels[0]))
    f = rs.factor_subdomain(O, part, sd, tol, 64, sketch_seed=5, sub=0, rank_pred=pred)
    assert f.sketched > 0
    if scale == 1.0:
        assert f.sketched_pred > 0      # the rank-sized sketch was accepted
    g = sd.index
    worst = 0.0
    for b in f.levels[0]:
        p = np.concatenate([b.sk, b.rd])
        far = np.setdiff1d(np.arange(len(g)), p)
        Ysk, Yrd = O.block(g[far], g[b.sk]), O.block(g[far], g[b.rd])
        if len(b.rd):
            worst = max(worst, np.linalg.norm(Yrd - Ysk @ b.T) / np.linalg.norm(np.hstack([Ysk, Yrd])))
    print("worst relative far-field ID error", worst)
    assert worst <= 30 * tol

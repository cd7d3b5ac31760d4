"""Planted mistakes in the oracle must fail its CPU pins (CPU only, slow).

Each case copies oracle/ and the module's pin files to a temporary directory, plants one
plausible mistake in one oracle module (a dropped term, a flipped sign, a
wrong index, a transposed operand, a wrong constant), and runs that module's
pin files there.  The pins pass on the real oracle, so each run must fail.

Left out on purpose, being equivalent: the sign of the Householder vector in
the CPQR (either sign gives a valid reflector, and T = R11^{-1} R12, the pivots
and the ranks do not depend on it; only the rounding does), and the value the
FFT product's periodic kernel takes at offset n (an output point inside the grid
never reaches it: i - j stays within [-(n-1), n-1]).
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTANTS = [
    # (module, pin files, original text, planted text)
    ("ie.py", ["test_oracle_ie.py"], "return -np.log(r) / (2.0 * np.pi)", "return np.log(r) / (2.0 * np.pi)"),
    ("ie.py", ["test_oracle_ie.py"], "return 1.0 / (4.0 * np.pi * r)", "return 1.0 / (2.0 * np.pi * r)"),
    ("ie.py", ["test_oracle_ie.py"], "(np.log(h) - 0.5 * np.log(2.0) - 1.5 + np.pi / 4.0)",
     "(np.log(h) + 0.5 * np.log(2.0) - 1.5 + np.pi / 4.0)"),
    ("ie.py", ["test_oracle_ie.py"], "(np.log(2.0 + np.sqrt(3.0)) - np.pi / 6.0)",
     "(np.log(2.0 + np.sqrt(3.0)) - np.pi / 3.0)"),
    ("ie.py", ["test_oracle_ie.py"], "x1 = (np.arange(n, dtype=np.float64) + 0.5) / n",
     "x1 = (np.arange(n, dtype=np.float64) + 0.5) / (n + 1)"),
    ("ie.py", ["test_oracle_ie.py"], "return np.stack([a.transpose().reshape(-1) for a in axes], axis=1)",
     "return np.stack([a.reshape(-1) for a in axes], axis=1)"),
    ("ie.py", ["test_oracle_ie.py"], "self.weight = self.h ** d", "self.weight = self.h ** (d - 1)"),
    ("ie.py", ["test_oracle_ie.py"], "return self.b[rows][:, None] * a * self.c[cols][None, :]",
     "return self.b[rows][:, None] * a * self.b[cols][None, :]"),
    ("ie.py", ["test_oracle_ie.py"], "return self.b * self.c * self.a_self", "return self.b * self.a_self"),
    ("cpqr.py", ["test_oracle_cpqr.py"], "cand = int(np.nonzero(norms >= mx - tie * nu0)[0][0])",
     "cand = int(np.nonzero(norms >= mx - tie * nu0)[0][-1])"),
    ("cpqr.py", ["test_oracle_cpqr.py"], "if mx <= tol * nu0:", "if mx < tol * nu0 * 0.5:"),
    ("cpqr.py", ["test_oracle_cpqr.py"], "norms = np.sqrt(np.sum(A[j:, j:] ** 2, axis=0))",
     "norms = np.sqrt(np.sum(A[:, j:] ** 2, axis=0))"),
    ("cpqr.py", ["test_oracle_cpqr.py"], "perm[[j, piv]] = perm[[piv, j]]", "pass"),
    ("cpqr.py", ["test_oracle_cpqr.py"], "A[j:, j:] -= 2.0 * np.outer(v, v @ A[j:, j:])",
     "A[j:, j:] -= 1.0 * np.outer(v, v @ A[j:, j:])"),
    ("rs.py", ["test_oracle_rs.py"], "Brr = Arr - Ars @ T - T.T @ Asr + T.T @ Ass @ T",
     "Brr = Arr - Ars @ T + T.T @ Ass @ T"),
    ("rs.py", ["test_oracle_rs.py"], "Bsr = Asr - Ass @ T", "Bsr = Asr + Ass @ T"),
    ("rs.py", ["test_oracle_rs.py"], 'E = solve_triangular(G, Bsr.T, trans="T", lower=False).T',
     'E = solve_triangular(G, Bsr.T, trans="N", lower=False).T'),
    ("rs.py", ["test_oracle_rs.py"], "return G, E, Ass - E @ E.T", "return G, E, Ass + E @ E.T"),
    ("rs.py", ["test_oracle_rs.py"], "vr = v[b.rd] - b.T.T @ v[b.sk]", "vr = v[b.rd] + b.T.T @ v[b.sk]"),
    ("rs.py", ["test_oracle_rs.py"], "v[b.sk] -= b.T @ vr", "v[b.sk] += b.T @ vr"),
    ("rs.py", ["test_oracle_rs.py"], "z[sd.index] += self.apply_sub(i, R[sd.index])",
     "z[sd.index] = self.apply_sub(i, R[sd.index])"),
    ("rs.py", ["test_oracle_rs.py"], "Yp = ie.kernel(d, np.sqrt(np.sum(diff * diff, axis=2))) * w[None, :]",
     "Yp = ie.kernel(d, np.sqrt(np.sum(diff * diff, axis=2)))"),
    ("rs.py", ["test_oracle_rs.py"], "return np.vstack([Yn, Yp]), near", "return Yp, near"),
    ("rs.py", ["test_oracle_rs.py"], "mat[blk] = lvl[ca].Bss", "mat[blk] = prob.block(gidx[sks[a]], gidx[sks[a]])"),
    ("rs.py", ["test_oracle_rs.py"], "phi = j * (np.pi * (3.0 - np.sqrt(5.0)))", "phi = j * 0.05"),
    ("rs.py", ["test_oracle_rs.py"], "z = 1.0 - (2.0 * j + 1.0) / n_pxy", "z = 1.0 - (j + 0.5) / n_pxy"),
    ("rs.py", ["test_oracle_rs.py"], "alive[np.isin(allact, p[pr])] = False", "pass"),
    ("fftmv.py", ["test_oracle_fftmv.py"], "v = (prob.c * Xc[:, c]).reshape(shape)", "v = Xc[:, c].reshape(shape)"),
    ("fftmv.py", ["test_oracle_fftmv.py"], "Y[:, c] = prob.b * y + prob.b * prob.c * prob.a_self * Xc[:, c]",
     "Y[:, c] = prob.b * y + prob.b * prob.b * prob.a_self * Xc[:, c]"),
    ("sketch.py", ["test_oracle_sketch.py"], "z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)",
     "z = (z ^ (z >> np.uint64(31))) * np.uint64(0xBF58476D1CE4E5B9)"),
    ("sketch.py", ["test_oracle_sketch.py"], "if k <= ell - OVER:", "if k <= ell:"),
    ("sketch.py", ["test_oracle_sketch.py"], "ell = (3 * n + 4) // 5 + OVER", "ell = (n + 4) // 5 + OVER"),
    ("sketch.py", ["test_oracle_sketch.py"], "return 1.0 - 2.0 * top.astype(np.float64)",
     "return 1.0 - top.astype(np.float64)"),
    ("sketch.py", ["test_oracle_sketch.py"], "x = base + i * np.uint64(G2) + r * np.uint64(G3)",
     "x = base + i * np.uint64(G2) + r * np.uint64(0)"),
    ("dd.py", ["test_oracle_dd.py", "test_oracle_tables.py"], "color = sum((k[t] % 2) << t for t in range(d))",
     "color = sum((k[t] % 2) for t in range(d))"),
    ("dd.py", ["test_oracle_dd.py", "test_oracle_tables.py"],
     "lo = [max(0, k[t] * s - delta) for t in range(d)]\n"
     "                hi = [min(n, (k[t] + 1) * s + delta) for t in range(d)]\n                regions_of[color]",
     "lo = [max(0, k[t] * s) for t in range(d)]\n"
     "                hi = [min(n, (k[t] + 1) * s + delta) for t in range(d)]\n                regions_of[color]"),
    ("mlp.py", ["test_oracle_mlp.py"], "u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000",
     "u = (u + 0x8000) & 0xFFFF0000"),
    ("mlp.py", ["test_oracle_mlp.py"], "dz2 = np.outer(dy, W3) * (z2 > 0)", "dz2 = np.outer(dy, W3)"),
    ("mlp.py", ["test_oracle_mlp.py"], "dz1 = (dz2 @ W2) * (z1 > 0)", "dz1 = (dz2 @ W2.T) * (z1 > 0)"),
    ("mlp.py", ["test_oracle_mlp.py"], "dy = 2.0 * r / n", "dy = 2.0 * r"),
    ("mlp.py", ["test_oracle_mlp.py"], "vh = v / (1 - b2 ** step)", "vh = v"),
    ("mlp.py", ["test_oracle_mlp.py"], "return p - lr * mh / (np.sqrt(vh) + eps), m, v",
     "return p - lr * mh / np.sqrt(vh + eps), m, v"),
    ("mlp.py", ["test_oracle_mlp.py"], "m = b1 * m + (1 - b1) * g", "m = b1 * m + g"),
    ("precond.py", ["test_oracle_tables.py"],
     "Minv[np.ix_(sd.index, sd.index)] += cho_solve(fc, np.eye(len(sd.index)))",
     "Minv[np.ix_(sd.index, sd.index)] = cho_solve(fc, np.eye(len(sd.index)))"),
    ("precond.py", ["test_oracle_tables.py"], "z[sd.index] += cho_solve(fc, r[sd.index])",
     "z[sd.index] = cho_solve(fc, r[sd.index])"),
    ("precond.py", ["test_oracle_tables.py"], "S = L.T @ Minv @ L", "S = L @ Minv @ L.T"),
    ("pcg.py", ["test_oracle_pcg.py"], "p[:, act] = znew + beta * p[:, act]", "p[:, act] = znew - beta * p[:, act]"),
    ("pcg.py", ["test_oracle_pcg.py"], "beta = rznew / rz[act]", "beta = np.sum(r[:, act] * z[:, act], axis=0) / rz[act]"),
    ("pcg.py", ["test_oracle_pcg.py"], "z[:, act] = znew", "pass"),
    ("pcg.py", ["test_oracle_pcg.py"], "alpha = rz[act] / np.sum(p[:, act] * q, axis=0)",
     "alpha = np.sum(r[:, act] ** 2, axis=0) / np.sum(p[:, act] * q, axis=0)"),
]


def _run_one(base, idx, module, pins, orig, planted):
    d = os.path.join(base, "m%02d" % idx)
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(d, "oracle"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    os.makedirs(os.path.join(d, "tests"))
    for f in ["conftest.py"] + pins:
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(d, "tests", f))
    for x in ("synth", "pytest.ini", os.path.join("tests", "golden")):
        os.symlink(os.path.join(ROOT, x), os.path.join(d, x))
    path = os.path.join(d, "oracle", module)
    src = open(path).read()
    assert src.count(orig) == 1, (module, orig)
    open(path, "w").write(src.replace(orig, planted))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not slow"] +
                       ["tests/" + p for p in pins], capture_output=True, text=True, cwd=d, timeout=600,
                       env=dict(os.environ, OMP_NUM_THREADS="2", OPENBLAS_NUM_THREADS="2"))
    return r.returncode, r.stdout[-300:]


@pytest.mark.slow
def test_every_planted_mistake_fails_a_pin(tmp_path):
    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as ex:
        futs = [ex.submit(_run_one, str(tmp_path), i, *m) for i, m in enumerate(MUTANTS)]
        results = [f.result() for f in futs]
    survived = [(MUTANTS[i][0], MUTANTS[i][3]) for i, (rc, _) in enumerate(results) if rc == 0]
    assert not survived, survived
    # a failing run must be a failed pin, not a broken copy (exit status 1: tests failed)
    assert all(rc == 1 for rc, _ in results), [out for rc, out in results if rc != 1]

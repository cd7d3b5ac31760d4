"""Write the stored FP64 oracle solution used by the full-size GPU solution tests.

Calls only oracle/ and synth/.  Workload: the 2D 512^2 cell-centred grid
(N = 262144), b = c = 1 + 0.5 sin(2 pi x1) cos(2 pi x2), CBD with 64^2
partitions and overlap 1 (4 subdomains), RS factors with ID tolerance 1e-6 and
64 proxy points at 1.5 box sides, right-hand side column 0 of
default_rng(0).standard_normal((nrhs, N)).  The oracle solves A u = f by PCG
(Section 5) with its FP64 RS preconditioner and the FFT product to relative
residual 1e-12, and stores u as float64 .npy beside a JSON record of how it
was made (iterations, recurrence and true residuals, and the distance of the
oracle's own 1e-10 iterate from the stored solution).

    python3 tests/golden/make_solution_fixture.py [--n 512]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import dd, fftmv, ie, pcg, rs  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--m", type=int, default=None, help="partitions per axis (default n/8)")
    args = ap.parse_args()
    n = args.n
    m = args.m or n // 8
    d, tol, npxy = 2, 1e-6, 64
    N = n ** d
    coef = synth.coef_smooth(d, n)
    prob = ie.Problem(d, n, b=coef, c=coef)
    part = dd.Partition(d, n, m, 1, dd.CBD)
    t0 = time.time()
    M = rs.RSPreconditioner(prob, part, tol, n_pxy=npxy, proxy_ratio=1.5)
    t_factor = time.time() - t0
    print("oracle RS factor: %.1f s, S = %s" % (t_factor, [s["S"] for s in M.stats()]), flush=True)
    A = fftmv.FFTMatvec(prob)
    f = synth.rhs(N, 1, seed=0)[0]
    t0 = time.time()
    u, it, rr = pcg.pcg(A, M.apply, f, tol=1e-12, maxit=400)
    t_pcg = time.time() - t0
    true_res = float(np.linalg.norm(f - A(u)) / np.linalg.norm(f))
    print("oracle PCG to 1e-12: %d iterations, %.1f s, true residual %.2e" % (it, t_pcg, true_res), flush=True)
    u10, it10, rr10 = pcg.pcg(A, M.apply, f, tol=1e-10, maxit=400)
    gap10 = float(np.linalg.norm(u10 - u) / np.linalg.norm(u))
    print("oracle PCG to 1e-10: %d iterations, distance to the 1e-12 solution %.2e" % (it10, gap10), flush=True)
    name = "u_%dsq_cbd_col0" % n
    np.save(os.path.join(HERE, name + ".npy"), u)
    rec = {
        "about": "FP64 oracle solution of A u = f (Section 2.1; PCG of Section 5 with the RS preconditioner "
                 "of Section 4.2 and the FFT product), written by tests/golden/make_solution_fixture.py",
        "d": d, "n": n, "m": m, "delta": 1, "mode": "cbd", "coef": "1+0.5 sin(2 pi x1) cos(2 pi x2)",
        "rs_tol": tol, "n_pxy": npxy, "proxy_ratio": 1.5, "rhs": "synth.rhs(N, nrhs, seed=0)[0]",
        "pcg_tol": 1e-12, "iterations": int(it), "recurrence_relres": float(rr), "true_relres": true_res,
        "oracle_1e-10_iterations": int(it10), "oracle_1e-10_rel_distance": gap10,
        "u_norm": float(np.linalg.norm(u)), "S": [s["S"] for s in M.stats()],
        "factor_s": t_factor, "pcg_s": t_pcg,
    }
    with open(os.path.join(HERE, name + ".json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()

"""Benchmark of the CBD-RS-PCG hot path on one MI355X.

Workload (2D, 512^2 grid, N = 262144): Laplace first-kind IE with smooth
coefficients b = c = 1 + 0.5 sin(2 pi x1) cos(2 pi x2); CBD decomposition with
64^2 partitions, overlap 1 (4 subdomains); RS factors with ID tolerance 1e-6 and
64 proxy points at 1.5 box sides; 64 right-hand sides f ~ N(0,1) (seed 0);
PCG to relative residual 1e-10.

One step = the whole hot path on resident inputs: RS factorization of all
subdomains (mixed form: FP64 ID, FP32 elimination/storage/apply) + PCG on the
64 right-hand sides at once (FP64 matvec and recurrences).  `value` is the PCG
solve time of one step in seconds.  After the timed steps, the plain FP64 form
(FP64 factors, one right-hand side at a time) is timed on a few columns and
scaled to 64, and the oracle's dense matvec is timed on sampled rows for the
CPU baseline.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PCG solve time (s) & RS factor GFLOP/s at 2D 512^2, mixed vs FP64, rel res 1e-10"

# The workloads (cell-centred grids, Laplace kernel, closed-form diagonal, PCG to 1e-10).
# "512sq" is the default measured configuration; the others are selectable with --workload.
WORKLOADS = {
    "64sq": dict(d=2, n=64, m=16, mode="cbd", delta=1, leaf=0, tol=1e-8, npxy=64, nrhs=1,
                 prec="fp64", coef=False, label="2D 64^2, CBD m=16, tol 1e-8, 1 RHS, FP64"),
    "256sq": dict(d=2, n=256, m=4, mode="schwarz", delta=8, leaf=8, tol=1e-6, npxy=64, nrhs=1,
                  prec="fp64", coef=False,
                  label="2D 256^2, Schwarz 4x4 subdomains, overlap one 8x8 leaf, tol 1e-6, 1 RHS, FP64"),
    "512sq": dict(d=2, n=512, m=64, mode="cbd", delta=1, leaf=0, tol=1e-6, npxy=64, nrhs=64,
                  prec="fp32", coef=True,
                  label="2D 512^2 (N=262144), b=c=1+0.5sin(2pi x1)cos(2pi x2), CBD m=64 delta=1, "
                        "RS tol 1e-6, 64 proxy pts at 1.5 box sides, 64 RHS N(0,1) seed 0, PCG rel res 1e-10"),
    "32cube": dict(d=3, n=32, m=8, mode="cbd", delta=1, leaf=0, tol=1e-6, npxy=256, nrhs=16,
                   prec="fp32", coef=False,
                   label="3D 32^3, CBD m=8 (8 subdomains), tol 1e-6, 256 proxy pts, 16 RHS, FP32 factors"),
    "1024sq": dict(d=2, n=1024, m=128, mode="cbd", delta=1, leaf=0, tol=1e-6, npxy=64, nrhs=1,
                   prec="fp32", coef=False,
                   label="2D 1024^2 (N=1048576), CBD m=128, tol 1e-6, 1 RHS, FP32 factors with the rank predictor"),
    # the paper's comparison system: global RS, one non-overlapping subdomain (the whole grid)
    # 3D at the paper's weak-scaling layout (N/M = 512 points per partition) and its
    # tolerance (1e-3), with randomized IDs as in the paper's last 3D runs
    "64cube": dict(d=3, n=64, m=8, mode="cbd", delta=1, leaf=0, tol=1e-3, npxy=256, nrhs=16,
                   prec="fp32", coef=False, sketch=True,
                   label="3D 64^3 (N=262144), CBD m=8 (N/M=512), tol 1e-3, 256 proxy pts, sketched IDs, "
                         "16 RHS, FP32 factors"),
    "128cube": dict(d=3, n=128, m=16, mode="cbd", delta=1, leaf=0, tol=1e-3, npxy=256, nrhs=1,
                    prec="fp32", coef=False, sketch=True, fft=True,
                    label="3D 128^3 (N=2097152), CBD m=16 (N/M=512), tol 1e-3, 256 proxy pts, sketched IDs, "
                          "1 RHS, FP32 factors, FFT matvec in PCG"),
    "256cube": dict(d=3, n=256, m=32, mode="cbd", delta=1, leaf=0, tol=1e-3, npxy=256, nrhs=1,
                    prec="fp32", coef=False, sketch=True, fft=True, dense=False, variants=False,
                    label="3D 256^3 (N=16777216), CBD m=32 (N/M=512), tol 1e-3, 256 proxy pts, sketched IDs, "
                          "1 RHS, FP32 factors, FFT matvec in PCG (no dense product: 2.8e14 pairs)"),
    # the paper's own 512^2 row of its 2D weak-scaling table: tolerance 1e-3, constant
    # coefficients, one right-hand side, FFT products, FP64 factors, PCG to 1e-12
    "512sq_paper": dict(d=2, n=512, m=64, mode="cbd", delta=1, leaf=0, tol=1e-3, npxy=64, nrhs=1,
                        prec="fp64", coef=False, fft=True, dense=False, variants=False, pcg_tol=1e-12,
                        label="2D 512^2 at the paper's settings: CBD m=64, tol 1e-3, b=c=1, FP64 factors, "
                              "1 RHS, FFT products, PCG to 1e-12"),
    "global512": dict(d=2, n=512, m=1, mode="jacobi", delta=0, leaf=8, tol=1e-6, npxy=64, nrhs=64,
                      prec="fp32", coef=True,
                      label="2D 512^2, global RS (one subdomain, 8x8 leaf tiles), b=c=1+0.5sin(2pi x1)cos(2pi x2), "
                            "tol 1e-6, 64 proxy pts, 64 RHS, FP32 factors"),
}
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector (and matrix) peak
FP32_PEAK_TFLOPS = 157.3


def measured_traffic(shape):
    """HBM bytes per launch of the 512^2 64-RHS matvec from the committed rocprofv3
    counter summary, or None if the kernel source changed since it was taken or the
    counters were taken for another tile shape."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "kernel_matvec_2d_512sq_64rhs.traffic.json")
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if hashlib.sha256(src).hexdigest() != rec.get("source_sha256") or rec.get("shape") != shape:
        return None
    return rec["traffic_bytes"]


def oracle_solution(args_workload, n):
    """The stored FP64 oracle solution of column 0 (tests/golden), written by
    tests/golden/make_solution_fixture.py from the oracle's RS-PCG to 1e-12; None for
    workloads without one."""
    import numpy as np
    if args_workload != "512sq":
        return None
    path = os.path.join(ROOT, "tests", "golden", "u_%dsq_cbd_col0.npy" % n)
    return np.load(path) if os.path.exists(path) else None


# Layouts whose ranks train the rank predictor: a mixed stream of 2D grids from 128^2 to
# 512^2 (N/M = 64, tol 1e-6), the 64^2 (tol 1e-8) and 256^2 Schwarz workloads, and 3D
# grids at the paper's 3D layout (N/M = 512, tol 1e-3) and at tol 1e-6.
# (d, n, m, mode, delta, leaf, tol, n_pxy)
TRAIN_LAYOUTS = [(2, 128, 16, "cbd", 1, 0, 1e-6, 64), (2, 192, 24, "cbd", 1, 0, 1e-6, 64),
                 (2, 256, 32, "cbd", 1, 0, 1e-6, 64), (2, 320, 40, "cbd", 1, 0, 1e-6, 64),
                 (2, 384, 48, "cbd", 1, 0, 1e-6, 64), (2, 448, 56, "cbd", 1, 0, 1e-6, 64),
                 (2, 512, 64, "cbd", 1, 0, 1e-6, 64), (2, 64, 16, "cbd", 1, 0, 1e-8, 64),
                 (2, 256, 4, "schwarz", 8, 8, 1e-6, 64), (3, 16, 4, "cbd", 1, 0, 1e-6, 256),
                 (3, 24, 3, "cbd", 1, 0, 1e-3, 256), (3, 32, 4, "cbd", 1, 0, 1e-3, 256)]
# held out: 2D 1024^2 (N/M = 64, tol 1e-6) and 3D 48^3 (N/M = 512, tol 1e-3)
HELD_OUT = [(2, 1024, 128, "cbd", 1, 0, 1e-6, 64), (3, 48, 6, "cbd", 1, 0, 1e-3, 256)]


def layout_ranks(cbd, dev, lay):
    d, n, m, mode, delta, leaf, tol, npxy = lay
    mode = {"cbd": cbd.MODE_CBD, "schwarz": cbd.MODE_SCHWARZ, "jacobi": cbd.MODE_JACOBI}[mode]
    Pt = cbd.Problem(d, n, device=dev)
    Ft = cbd.Factor(Pt, cbd.Partition(Pt, m, delta, mode, leaf), tol=tol, n_pxy=npxy, precision=cbd.PREC_FP32)
    return Ft.all_features()


def train_rank_predictor(cbd, dev):
    """Skeleton-rank MLP trained by the library's kernels on (features, rank) pairs of
    TRAIN_LAYOUTS' factorizations; returns the network and its held-out rank errors."""
    import numpy as np
    Xs, ks = [], []
    for lay in TRAIN_LAYOUTS:
        X, k = layout_ranks(cbd, dev, lay)
        Xs.append(X)
        ks.append(k)
    rng = np.random.default_rng(0)
    H, F = 64, cbd.RankMLP.F
    p0 = np.concatenate([rng.standard_normal(H * F) * np.sqrt(2.0 / F), np.zeros(H),
                         rng.standard_normal(H * H) * np.sqrt(2.0 / H), np.zeros(H),
                         rng.standard_normal(H) * np.sqrt(1.0 / H), np.zeros(1)]).astype(np.float32)
    net = cbd.RankMLP(p0, dev)
    net.train(np.concatenate(Xs), np.concatenate(ks), steps=1500, lr=1e-2)
    held = {}
    for lay in HELD_OUT:
        X, k = layout_ranks(cbd, dev, lay)
        kp = net.predict_ranks(X).cpu().numpy()
        held["%dd_%d" % (lay[0], lay[1])] = {"boxes": int(len(k)), "mean_k": float(np.mean(k)),
                                            "mean_abs_err": float(np.mean(np.abs(kp - k)))}
    return net, held


# Size series for the complexity study of Section 4.4: (n, m) pairs.  "sublinear": m
# is the divisor of n closest (in log) to n^(6/7) in 2D (M ~ N^(6/7)) or n^(3/4) in 3D
# (M ~ N^(3/4)), the partition counts of the corollary th:optimal; "fixed": N/M = 64
# (2D) and 512 (3D), the layouts of the paper's weak-scaling tables.  Settings of those
# tables: tol 1e-3, b = c = 1, FP64 factors, FFT products, PCG to 1e-10.
SERIES = {
    "2d": dict(d=2, npxy=64, sublinear=[(120, 60), (240, 120), (480, 240), (960, 320), (1920, 640)],
               fixed=[(128, 16), (256, 32), (512, 64), (1024, 128), (2048, 256)],
               theory={"sublinear": {"t_f": 9 / 7, "m_f": 8 / 7}}),
    "3d": dict(d=3, npxy=256, sublinear=[(16, 8), (24, 12), (32, 16), (48, 16), (96, 32)],
               fixed=[(32, 4), (64, 8), (128, 16)],
               theory={"sublinear": {"t_f": 3 / 2, "m_f": 5 / 4}}),
}


def id_method(cbd, choice, tol):
    """CBD_ID_GRAM for choice "gram", or "auto" when tol >= 1e-7; else CBD_ID_QR."""
    if choice == "gram" or (choice == "auto" and tol >= 1e-7):
        return cbd.ID_GRAM
    return cbd.ID_QR


def run_series(kind, id_choice="auto"):
    """One JSON line: per size N, M, S, t_f, m_f, n_it, t_pcg for both layouts, and the
    least-squares exponents of t_f and m_f against N."""
    import numpy as np
    import torch

    import paper_2108_12574_amd as cbd
    import synth

    dev = torch.device("cuda:0")
    cfg = SERIES[kind]
    d = cfg["d"]
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    out = {"series": kind, "settings": "CBD, overlap 1, tol 1e-3, %d proxy points, b = c = 1, FP64 factors, "
                                      "1 RHS f ~ N(0,1) seed 0, FFT products, PCG to 1e-10" % cfg["npxy"],
           "id_method": "gram" if id_method(cbd, id_choice, 1e-3) == cbd.ID_GRAM else "qr",
           "theory": cfg["theory"], "rows": {}, "fit": {}}
    for layout in ("sublinear", "fixed"):
        rows = []
        for n, m in cfg[layout]:
            N = n ** d
            P = cbd.Problem(d, n, device=dev)
            part = cbd.Partition(P, m, 1, cbd.MODE_CBD, 0)
            f = torch.tensor(synth.rhs(N, 1, seed=0), device=dev)
            P.fft_prepare(max_pairs=1)
            opts = dict(tol=1e-3, n_pxy=cfg["npxy"], proxy_ratio=1.5, precision=cbd.PREC_FP64, apply_rhs=1,
                        sketch_seed=1 if d == 3 else None, id_method=id_method(cbd, id_choice, 1e-3))
            fac = cbd.Factor(P, part, **opts)            # warm-up; sizes the workspace
            hint, ws = fac.ranks.cpu(), fac.ws
            del fac
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fac = cbd.Factor(P, part, rank_hint=hint, ws=ws, **opts)
            torch.cuda.synchronize()
            t_f = time.perf_counter() - t0
            t0 = time.perf_counter()
            u, it, rr = cbd.pcg_solve(P, fac, f[0], tol=1e-10, maxit=300, fft=True)
            torch.cuda.synchronize()
            t_pcg = time.perf_counter() - t0
            st = fac.stats()
            row = {"n": n, "m": m, "N": N, "M": m ** d, "S_max": max(st["S"]), "t_f": t_f,
                   "m_f_bytes": st["bytes"], "flops": st["flops"], "n_it": it, "relres": rr, "t_pcg": t_pcg}
            log(layout, row)
            rows.append(row)
            del fac, u, P, part
            torch.cuda.empty_cache()
        out["rows"][layout] = rows
        lN = np.log([r["N"] for r in rows])
        out["fit"][layout] = {q: float(np.polyfit(lN, np.log([r[k] for r in rows]), 1)[0])
                              for q, k in (("t_f", "t_f"), ("m_f", "m_f_bytes"), ("flops", "flops"),
                                           ("M", "M"))}
    print(json.dumps(out))


def library_dgemm_tflops(dev, n=8192, reps=3):
    """FP64 TFLOP/s of the vendor library's GEMM (torch.matmul) on n x n operands: the
    rate FP64 matrix-core code reaches on this GPU in practice, beside the nominal peak."""
    import torch
    a = torch.randn(n, n, dtype=torch.float64, device=dev)
    b = torch.randn(n, n, dtype=torch.float64, device=dev)
    c = a @ b
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        c = a @ b
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    del a, b, c
    return 2.0 * n ** 3 / t / 1e12


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and the cores this process may use."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return name, cores


def oracle_rs_sample(fac, O, opart, tol, npxy, nrhs, per_level=4):
    """The oracle's RS factorization and apply timed on sampled boxes and scaled by the
    box counts.  For every compressed level, per_level boxes of subdomain 0 (drawn
    with a fixed seed) take the oracle's steps with the GPU factor's active DOFs: the proxy matrix
    (oracle.rs.proxy_matrix, near field from the level's other active DOFs), the ID
    (oracle.cpqr.interp_decomp), the elimination (oracle.rs.eliminate_box, with the
    kernel block of the box's DOFs standing in for its Schur-complement block: same
    sizes and flops), and the forward and backward sweep steps of the apply on nrhs
    columns; each level's mean per box is scaled by its boxes over all subdomains.
    The roots: a Cholesky factorization and a solve of each subdomain's root size.
    Returns (factor_s, apply_s, detail)."""
    import numpy as np
    from scipy.linalg import cho_factor, cho_solve
    from oracle import rs
    from oracle.cpqr import interp_decomp
    rng = np.random.default_rng(0)
    nlev = fac.stats()["levels"]
    t_fac = t_app = 0.0
    detail = []
    sd = opart.subdomains[0]
    for l in range(min(nlev, sd.root_level)):
        total = len(fac.level(l)[0])                       # boxes of the level, all subdomains
        boxes = [fac.box(0, l, b) for b in range(len(sd.levels[l]))]
        act = [np.concatenate([g["sk"], g["rd"]]).astype(np.int64) for g in boxes]
        allact = np.concatenate(act)
        pick = np.sort(rng.choice(len(boxes), min(per_level, len(boxes)), replace=False))
        tf = ta = 0.0
        for b in pick:
            p = act[b]
            t0 = time.perf_counter()
            Y, _ = rs.proxy_matrix(O, sd, sd.levels[l][b], p, np.setdiff1d(allact, p), npxy)
            k, perm, T = interp_decomp(Y, tol)
            G, E, Bss = rs.eliminate_box(O.block(sd.index[p], sd.index[p]), perm[:k], perm[k:], T)
            t1 = time.perf_counter()
            bf = rs.BoxFactor(perm[:k], perm[k:], T, G, E, Bss)
            v = rng.standard_normal((len(p), nrhs))
            t2 = time.perf_counter()
            rs.box_forward(bf, v)
            rs.box_backward(bf, v)
            t3 = time.perf_counter()
            tf += t1 - t0
            ta += t3 - t2
        tf, ta = tf / len(pick) * total, ta / len(pick) * total
        t_fac += tf
        t_app += ta
        detail.append({"level": l, "boxes": total, "sampled": int(len(pick)), "factor_s": tf, "apply_s": ta})
    for i in range(len(opart.subdomains)):
        S = fac.stats()["S"][i]
        if S == 0:
            continue
        idx = fac.root(i)[0]
        A = O.block(opart.subdomains[i].index[idx], opart.subdomains[i].index[idx])
        t0 = time.perf_counter()
        c = cho_factor(A)
        t1 = time.perf_counter()
        cho_solve(c, rng.standard_normal((S, nrhs)))
        t2 = time.perf_counter()
        t_fac += t1 - t0
        t_app += t2 - t1
    detail.append({"roots": len(opart.subdomains)})
    return t_fac, t_app, detail


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="512sq", choices=sorted(WORKLOADS))
    ap.add_argument("--fp64-cols", type=int, default=8,
                    help="columns solved one at a time to time the plain FP64 form")
    ap.add_argument("--factor-only", action="store_true",
                    help="run one factorization of the workload (no predictor, no PCG) and print its time; "
                         "for counter profiles of the factor kernels")
    ap.add_argument("--matvec-only", action="store_true",
                    help="autotune the dense matvec, then run three products with the workload's right-hand "
                         "sides and three plain copies of as many doubles (the traffic counters' calibration); "
                         "for counter profiles of the matvec")
    ap.add_argument("--apply-only", action="store_true",
                    help="factor the workload once (no predictor), then run ten preconditioner applies on its "
                         "right-hand sides; for profiles of the apply")
    ap.add_argument("--cpu-rows", type=int, default=-1,
                    help="rows of the oracle's dense matvec timed for the CPU baseline (0: skip; "
                         "-1: about 12 s of host work, 16384 rows at 512^2 with 64 RHS)")
    ap.add_argument("--id", choices=["auto", "qr", "gram"], default="auto",
                    help="IDs of the levels of few, large boxes: column-pivoted Householder QR, or the pivoted "
                         "Cholesky of the Gram matrix (same ID in exact arithmetic; tol >= 1e-7); auto: gram "
                         "when the workload's tol allows it")
    ap.add_argument("--series", choices=sorted(SERIES),
                    help="instead of the benchmark line: factor and solve a series of grid sizes with the "
                         "partition count growing sublinearly (Section 4.4) and with N/M fixed, and fit "
                         "the exponents of t_f and m_f in N")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU only (--gpus 1); sharding the path over "
              "several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.series:
        run_series(args.series, args.id)
        return

    import numpy as np
    import torch

    import paper_2108_12574_amd as cbd
    import synth

    dev = torch.device("cuda:0")
    W = WORKLOADS[args.workload]
    d, n, nrhs, tol, npxy = W["d"], W["n"], W["nrhs"], W["tol"], W["npxy"]
    mode = {"cbd": cbd.MODE_CBD, "schwarz": cbd.MODE_SCHWARZ, "jacobi": cbd.MODE_JACOBI}[W["mode"]]
    prec = {"fp32": cbd.PREC_FP32, "fp64": cbd.PREC_FP64}[W["prec"]]
    sk_seed = 1 if W.get("sketch") else None      # randomized IDs
    use_fft = bool(W.get("fft"))                   # PCG products by FFT (workloads too large for the dense form)
    pcg_tol = W.get("pcg_tol", 1e-10)              # relative residual of the timed PCG
    dense = W.get("dense", True)                   # time the dense matvec (autotune, roofline)
    full = W.get("variants", True)                 # the variants (no predictor, FFT, sketch, bf16, FP64 form)
    idm = id_method(cbd, args.id, tol)
    N = n ** d
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    coef = torch.tensor(synth.coef_smooth(d, n)) if W["coef"] else None
    P = cbd.Problem(d, n, b=coef, c=coef, device=dev)
    part = cbd.Partition(P, W["m"], W["delta"], mode, W["leaf"])
    F_rhs = torch.tensor(synth.rhs(N, nrhs, seed=0), device=dev)
    torch.cuda.synchronize()

    if args.factor_only:
        cbd.timing.reset()
        cbd.timing.enable(True)
        t0 = time.perf_counter()
        fac = cbd.Factor(P, part, tol=tol, n_pxy=npxy, proxy_ratio=1.5, precision=prec, sketch_seed=sk_seed,
                         id_method=idm)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        cbd.timing.enable(False)
        t_gpu = cbd.timing.get("factor")[0] / 1e3
        st = fac.stats()
        sched = fac.schedule()
        # the same factorization recorded, captured as a graph and replayed five times
        replay = None
        if t_gpu < 1.0:
            del fac
            fac = cbd.Factor(P, part, tol=tol, n_pxy=npxy, proxy_ratio=1.5, precision=prec, sketch_seed=sk_seed,
                             id_method=idm, record=True)
            fac.capture()
            times = []
            for _ in range(5):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ok = fac.replay()
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
                assert ok
            replay = {"replay_s": min(times), "replay_s_all": times, "gflops": st["flops"] / min(times) / 1e9}
        print(json.dumps({"workload": W["label"], "factor_s": t, "factor_gpu_s": t_gpu,
                          "note": "factor_s includes sizing and allocating the workspace; factor_gpu_s is the "
                                  "factorization's launch sequence between HIP events on its stream; replay: "
                                  "the captured graph of the same factorization launched again (wall time, one "
                                  "synchronization each)",
                          "factor_flops": st["flops"], "factor_gflops": st["flops"] / t_gpu / 1e9,
                          "schedule": sched, "replay": replay}))
        return

    if args.apply_only:
        fac = cbd.Factor(P, part, tol=tol, n_pxy=npxy, proxy_ratio=1.5, precision=prec, sketch_seed=sk_seed,
                         id_method=idm, apply_rhs=nrhs)
        z = fac.apply(F_rhs)
        torch.cuda.synchronize()
        cbd.timing.reset()
        cbd.timing.enable(True)
        for _ in range(10):
            z = fac.apply(F_rhs)
        torch.cuda.synchronize()
        cbd.timing.enable(False)
        ms, cnt = cbd.timing.get("apply")
        # the same with the apply's columns per workgroup tuned level by level
        cols = fac.autotune_apply(F_rhs)
        z = fac.apply(F_rhs)
        torch.cuda.synchronize()
        cbd.timing.reset()
        cbd.timing.enable(True)
        for _ in range(10):
            z = fac.apply(F_rhs)
        torch.cuda.synchronize()
        cbd.timing.enable(False)
        ms_t, cnt_t = cbd.timing.get("apply")
        levels = []
        for l in range(fac.stats()["levels"] + 1):
            k, npl, _ = fac.level(l)
            levels.append({"level": l, "boxes": len(npl), "np_max": max(npl), "np_mean": float(np.mean(npl)),
                           "k_mean": float(np.mean(k))})
        print(json.dumps({"workload": W["label"], "apply_avg_ms": ms / max(cnt, 1),
                          "apply_tuned_ms": ms_t / max(cnt_t, 1), "apply_cols": cols,
                          "factor_bytes": fac.stats()["bytes"], "nrhs": nrhs, "levels": levels}))
        return

    if args.matvec_only:
        tile = P.autotune_matvec(nrhs)
        cbd.timing.reset()
        cbd.timing.enable(True)
        for _ in range(3):
            y = P.matvec(F_rhs)
        torch.cuda.synchronize()
        cbd.timing.enable(False)
        ms, cnt = cbd.timing.get("matvec")
        for _ in range(3):
            y.copy_(F_rhs)       # N x nrhs doubles read and written
        torch.cuda.synchronize()
        print(json.dumps({"workload": W["label"], "tile_shape": tile, "matvec_avg_ms": ms / max(cnt, 1),
                          "copy_bytes_each_way": 8 * N * nrhs, "library_dgemm_tflops": library_dgemm_tflops(dev)}))
        return

    P.fft_prepare(max_pairs=8)
    # tile shape of the matvec, chosen by the library's autotuner
    tile = P.autotune_matvec(nrhs) if dense else 0
    tile1 = P.autotune_matvec(1) if dense else 0
    log("matvec tile shape: %d (%d RHS), %d (1 RHS)" % (tile, nrhs, tile1))

    # rank predictor trained on ranks of a mixed stream of factorizations
    t0 = time.perf_counter()
    mlp, mlp_held = train_rank_predictor(cbd, dev)
    torch.cuda.synchronize()
    mlp_train_s = time.perf_counter() - t0
    log("rank predictor trained in %.2f s" % mlp_train_s)

    # The factor's device workspace and the PCG's are allocated once, before the timed
    # steps (sized by a first factorization), so that no step allocates device memory.
    fac0 = cbd.Factor(P, part, tol=tol, n_pxy=npxy, proxy_ratio=1.5, precision=prec, mlp=mlp, sketch_seed=sk_seed,
                      apply_rhs=nrhs, id_method=idm)
    used0 = fac0.ws_used
    del fac0                    # its own workspace goes before the timed steps' is allocated
    torch.cuda.empty_cache()
    ws_factor = torch.empty(int(used0 * 1.05) + (1 << 20), dtype=torch.uint8, device=dev)
    ws_pcg = cbd.pcg_workspace(P, nrhs)
    box = {"fac": None, "graph": False, "replay": False}
    side = torch.cuda.Stream(device=dev)    # PCG with captured HIP graphs needs a non-default stream

    def solve(fac, graph):
        if not graph:
            return cbd.pcg_solve(P, fac, F_rhs, tol=pcg_tol, maxit=200, fft=use_fft, ws=ws_pcg)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            out = cbd.pcg_solve(P, fac, F_rhs, tol=pcg_tol, maxit=200, fft=use_fft, ws=ws_pcg, graph=True)
        torch.cuda.current_stream(dev).wait_stream(side)
        return out

    def factor_step():
        t0 = time.perf_counter()
        # graph mode: the factorization of the previous step replayed from its captured graph
        # (every kernel runs again on the data; the host side is checked against the recording)
        if box["replay"] and box["fac"] is not None and box["fac"].captured and box["fac"].replay():
            fac = box["fac"]
        else:
            box["fac"] = None           # the previous factor views ws_factor: release it first
            fac = cbd.Factor(P, part, tol=tol, n_pxy=npxy, proxy_ratio=1.5, precision=prec, mlp=mlp,
                             sketch_seed=sk_seed, apply_rhs=nrhs, ws=ws_factor, id_method=idm, record=box["replay"])
            if box["replay"]:
                fac.capture()
            if box.get("apply_cols"):
                fac.set_apply_shapes(box["apply_cols"])
        torch.cuda.synchronize()
        box["fac"] = fac
        return fac, time.perf_counter() - t0

    def step():
        fac, t_fac = factor_step()
        t1 = time.perf_counter()
        u, its, rr = solve(fac, box["graph"])
        torch.cuda.synchronize()
        return fac, u, its, rr, t_fac, time.perf_counter() - t1

    # eager or graph-replayed PCG iterations: the faster one, measured once, runs the timed steps
    pcg_modes = {}
    for graph in (False, True):
        box["graph"] = graph
        pcg_modes["graph" if graph else "eager"] = step()[5]
    box["graph"] = pcg_modes["graph"] < pcg_modes["eager"]
    log("pcg eager %.3f s, graph %.3f s: timed steps use %s" % (pcg_modes["eager"], pcg_modes["graph"],
                                                                 "graphs" if box["graph"] else "eager launches"))
    # the factorization launched eagerly (host planning, a synchronization per rank read)
    # or replayed from a graph captured after an eager run: the faster one runs the timed steps
    # (factorizations of a second or more are left eager: launch overhead is no part of them)
    fac_modes = {"eager": min(factor_step()[1] for _ in range(2)), "graph": None}
    if fac_modes["eager"] < 1.0:
        box["replay"] = True
        factor_step()                   # eager, recorded, captured
        fac_modes["graph"] = min(factor_step()[1] for _ in range(2))
        box["replay"] = fac_modes["graph"] < fac_modes["eager"]
    # the apply's columns per workgroup, tuned level by level on the current factor (the
    # timed steps' factors take the same choices)
    box["apply_cols"] = box["fac"].autotune_apply(F_rhs)
    log("apply columns per workgroup by level: %s" % box["apply_cols"])
    log("factor eager %.4f s, graph replay %s s: timed steps use %s"
        % (fac_modes["eager"], "%.4f" % fac_modes["graph"] if fac_modes["graph"] else "-",
           "replays" if box["replay"] else "eager launches"))
    for w in range(args.warmup):
        step()
        log("warmup step %d done" % w)
    cbd.timing.reset()
    cbd.timing.enable(True)
    torch.cuda.synchronize()
    tf, ts, its_all, rr_all = [], [], [], []
    t_start = time.perf_counter()
    for k in range(args.steps):
        fac, u_main, its, rr, a, b = step()
        tf.append(a)
        ts.append(b)
        its_all.append(its)
        rr_all.append(max(rr))
        log("step %d: factor %.3f s, pcg %.3f s, iterations %d-%d" % (k, a, b, min(its), max(its)))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    cbd.timing.enable(False)
    mv_ms, mv_n = cbd.timing.get("matvec")
    ap_ms, ap_n = cbd.timing.get("apply")
    st = fac.stats()
    sched = fac.schedule()
    factor_s = float(np.mean(tf))
    # the same factorization without the predictor
    factor_nm_s, sched_nm = None, {"host_syncs": None}
    if full:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac_nm = cbd.Factor(P, part, tol=tol, n_pxy=npxy, proxy_ratio=1.5, precision=prec, sketch_seed=sk_seed,
                            id_method=idm)
        torch.cuda.synchronize()
        factor_nm_s = time.perf_counter() - t0
        sched_nm = fac_nm.schedule()
        del fac_nm
    # what the predictor gains on a sketched 3D factorization (64^3, N/M = 512, tol 1e-3):
    # rank-sized first sketches; same PCG iteration counts
    mlp_gain_3d = None
    if full:
        P3 = cbd.Problem(3, 64, device=dev)
        part3 = cbd.Partition(P3, 8, 1, cbd.MODE_CBD, 0)
        f3 = torch.tensor(synth.rhs(64 ** 3, 1, seed=0), device=dev)
        P3.fft_prepare(max_pairs=1)
        leg = {}
        for name, net in (("without", None), ("with", mlp)):
            times = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                F3 = cbd.Factor(P3, part3, tol=1e-3, n_pxy=256, precision=cbd.PREC_FP32, mlp=net, sketch_seed=1,
                                apply_rhs=1, id_method=id_method(cbd, args.id, 1e-3))
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            _, it3, _ = cbd.pcg_solve(P3, F3, f3[0], tol=1e-10, maxit=300, fft=True)
            sc3 = F3.schedule()
            leg[name] = {"factor_s": float(np.median(times)), "flops": F3.stats()["flops"], "n_it": it3,
                         "rank_sized_sketches": sc3["sketched_pred"], "sketched": sc3["sketched"]}
            del F3
        mlp_gain_3d = leg
        log("predictor on 3D 64^3: %s" % leg)
        del P3, part3, f3
    pcg_s = float(np.mean(ts))
    n_it = its_all[-1]
    u_ref = oracle_solution(args.workload, n)
    u_err = {}

    def uerr(name, u0):
        """|u - u_oracle| / |u_oracle| over all N entries of column 0."""
        if u_ref is not None:
            u0 = u0.double().cpu().numpy()
            u_err[name] = float(np.linalg.norm(u0 - u_ref) / np.linalg.norm(u_ref))

    uerr("mixed_batched", u_main[0])

    if mv_n == 0 and dense:
        # the PCG used FFT products or replayed graphs (no timer events inside a capture):
        # time three dense products for the roofline record
        cbd.timing.reset()
        cbd.timing.enable(True)
        for _ in range(3):
            P.matvec(F_rhs)
        torch.cuda.synchronize()
        cbd.timing.enable(False)
        mv_ms, mv_n = cbd.timing.get("matvec")
    # one product with a single right-hand side (the plain FP64 form's matvec)
    mv1_ms = None
    if dense:
        cbd.timing.reset()
        cbd.timing.enable(True)
        for _ in range(3):
            P.matvec(F_rhs[0])
        torch.cuda.synchronize()
        cbd.timing.enable(False)
        t1, n1 = cbd.timing.get("matvec")
        mv1_ms = t1 / max(n1, 1)
        cbd.timing.reset()
    # matvec roofline: product flops 2 N^2 nrhs per launch (kernel evaluations extra)
    mv_avg_s = mv_ms / 1e3 / mv_n if mv_n else None
    mv_flops = 2.0 * N * N * nrhs
    achieved = mv_flops / mv_avg_s / 1e12 if mv_avg_s else None

    pcg_fft_s, its_fft, rr_fft, sketched, bf16, alt_id = None, [0], [0.0], None, None, None
    f64_factor, f64_pcg, ncols, its64, f64_batched = None, None, 0, [], None
    if full:
        # the paper's matvec (FFT on the uniform grid) with the same factors, for comparison
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u_fft, its_fft, rr_fft = cbd.pcg_solve(P, fac, F_rhs, tol=1e-10, maxit=200, fft=True)
        torch.cuda.synchronize()
        pcg_fft_s = time.perf_counter() - t0
        uerr("fft_matvec", u_fft[0])
        del u_fft
        log("pcg with the FFT matvec: %.3f s, iterations %d-%d" % (pcg_fft_s, min(its_fft), max(its_fft)))

        # randomized IDs: the CPQR of a random-sign sketch of each proxy matrix (the scheme of
        # the paper's last 3D runs); same predictor, same PCG
        # (the better of two factorizations: the first may wait on device allocations)
        sk_times = []
        for _ in range(2):
            fac_sk = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fac_sk = cbd.Factor(P, part, tol=tol, n_pxy=npxy, proxy_ratio=1.5, precision=prec, mlp=mlp, sketch_seed=1,
                                id_method=idm)
            torch.cuda.synchronize()
            sk_times.append(time.perf_counter() - t0)
        sk_factor = min(sk_times)
        t0 = time.perf_counter()
        u_sk, its_sk, rr_sk = cbd.pcg_solve(P, fac_sk, F_rhs, tol=1e-10, maxit=200, fft=use_fft)
        torch.cuda.synchronize()
        uerr("sketched_id", u_sk[0])
        del u_sk
        sk_sched = fac_sk.schedule()
        sketched = {"factor_s": sk_factor, "factor_gflops": fac_sk.stats()["flops"] / sk_factor / 1e9,
                    "pcg_s": time.perf_counter() - t0, "n_it": [min(its_sk), max(its_sk)], "max_relres": max(rr_sk),
                    "sketched_boxes": sk_sched["sketched"], "fallback_boxes": sk_sched["sketch_fallbacks"]}
        del fac_sk
        log("sketched IDs: %s" % sketched)

        # the other route to the same IDs: column-pivoted Householder QR, as (e:id) states it,
        # when the timed steps take the pivoted Cholesky of the Gram matrix (or the reverse)
        alt_idm = cbd.ID_QR if idm == cbd.ID_GRAM else (cbd.ID_GRAM if tol >= 1e-7 else None)
        if alt_idm is not None:
            alt_name = "qr" if alt_idm == cbd.ID_QR else "gram"
            fac_alt = None
            tts = []
            for _ in range(2):
                del fac_alt
                fac_alt = None
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fac_alt = cbd.Factor(P, part, tol=tol, n_pxy=npxy, proxy_ratio=1.5, precision=prec, mlp=mlp,
                                     sketch_seed=sk_seed, apply_rhs=nrhs, id_method=alt_idm)
                torch.cuda.synchronize()
                tts.append(time.perf_counter() - t0)
            t0 = time.perf_counter()
            u_alt, its_alt, rr_alt = cbd.pcg_solve(P, fac_alt, F_rhs, tol=1e-10, maxit=200, fft=use_fft)
            torch.cuda.synchronize()
            alt_pcg = time.perf_counter() - t0
            uerr(alt_name + "_id", u_alt[0])
            del u_alt
            st_alt = fac_alt.stats()
            alt_id = {"id_method": alt_name, "factor_s": min(tts), "factor_gflops": st_alt["flops"] / min(tts) / 1e9,
                      "S_last_level": st_alt["S"], "pcg_s": alt_pcg, "n_it": [min(its_alt), max(its_alt)],
                      "max_relres": max(rr_alt), "host_syncs": fac_alt.schedule()["host_syncs"]}
            del fac_alt
            log("%s IDs: %s" % (alt_name, alt_id))

        # the bfloat16-GEMM variant of the factors (Schur products on bf16 operands)
        bf16 = None
        try:
            bf_times = []
            for _ in range(2):   # the better of two, as above
                fac_bf = None
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fac_bf = cbd.Factor(P, part, tol=tol, n_pxy=npxy, proxy_ratio=1.5, precision=cbd.PREC_BF16GEMM,
                                    mlp=mlp, sketch_seed=sk_seed, id_method=idm)
                torch.cuda.synchronize()
                bf_times.append(time.perf_counter() - t0)
            bf_factor = min(bf_times)
            t0 = time.perf_counter()
            u_bf, its_bf, rr_bf = cbd.pcg_solve(P, fac_bf, F_rhs, tol=1e-10, maxit=400, flexible=True,
                                                fft=use_fft)
            torch.cuda.synchronize()
            uerr("bf16_gemm_flexible", u_bf[0])
            del u_bf
            bf16 = {"factor_s": bf_factor, "pcg_s": time.perf_counter() - t0, "n_it": [min(its_bf), max(its_bf)],
                    "max_relres": max(rr_bf), "pcg": "flexible"}
            del fac_bf
        except cbd.CbdError as e:
            bf16 = {"error": str(e)}
        log("bf16-GEMM variant: %s" % bf16)

        # plain FP64 form: FP64 factors, right-hand sides one at a time
        f64_times = []
        for _ in range(2):   # the better of two, as above
            fac64 = None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fac64 = cbd.Factor(P, part, tol=tol, n_pxy=npxy, proxy_ratio=1.5, precision=cbd.PREC_FP64,
                               sketch_seed=sk_seed, id_method=idm)
            torch.cuda.synchronize()
            f64_times.append(time.perf_counter() - t0)
        f64_factor = min(f64_times)
        t0 = time.perf_counter()
        its64 = []
        ncols = min(args.fp64_cols, nrhs)
        for c in range(ncols):
            u64, it, _ = cbd.pcg_solve(P, fac64, F_rhs[c], tol=1e-10, maxit=200, fft=use_fft)
            its64.append(it)
            if c == 0:
                torch.cuda.synchronize()
                t_pause = time.perf_counter()
                uerr("fp64_one_column", u64)
                t0 += time.perf_counter() - t_pause     # the host-side comparison is not timed
        torch.cuda.synchronize()
        f64_per_col = (time.perf_counter() - t0) / max(ncols, 1)
        f64_pcg = f64_per_col * nrhs if ncols > 0 else float("nan")
        log("fp64 form: factor %.3f s, %.3f s per column" % (f64_factor, f64_per_col))
        # the same FP64 factors on all right-hand sides at once: separates what the
        # precision buys (FP32 vs FP64 factors, both batched) from what batching buys
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u64b, its64b, rr64b = cbd.pcg_solve(P, fac64, F_rhs, tol=1e-10, maxit=200, fft=use_fft)
        torch.cuda.synchronize()
        f64_batched = {"pcg_s": time.perf_counter() - t0, "n_it": [min(its64b), max(its64b)],
                       "max_relres": max(rr64b)}
        uerr("fp64_batched", u64b[0])
        del u64b
        log("fp64 factors, batched: %s" % f64_batched)

    dgemm_ref = library_dgemm_tflops(dev) if achieved else None
    cpu = None
    if args.cpu_rows < 0:
        # the row cost is proportional to N * nrhs
        args.cpu_rows = int(min(N, max(64, 16384.0 * (512 ** 2 * 64) / (float(N) * nrhs) / (4 if d == 3 else 1))))
    if args.cpu_rows > 0:
        from oracle import cmatvec, dd, ie
        O = ie.Problem(d, n, b=None if coef is None else coef.numpy(), c=None if coef is None else coef.numpy())
        rows = np.random.default_rng(0).choice(N, args.cpu_rows, replace=False)
        X = F_rhs.cpu().numpy().T.copy()
        t0 = time.perf_counter()
        cmatvec.matvec(O, X, rows=rows)
        t_rows = time.perf_counter() - t0
        per_matvec = t_rows * N / args.cpu_rows
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        model, avail = cpu_model()
        log("cpu baseline matvec sample %.2f s" % t_rows)
        # the oracle's RS factor and apply on sampled boxes (the PCG's other per-iteration step)
        omode = {"cbd": dd.CBD, "schwarz": dd.SCHWARZ, "jacobi": dd.JACOBI}[W["mode"]]
        opart = dd.Partition(d, n, W["m"], W["delta"], omode, W["leaf"])
        t0 = time.perf_counter()
        o_fac, o_app, o_detail = oracle_rs_sample(fac, O, opart, tol, npxy, nrhs)
        log("cpu baseline RS sample %.2f s: factor %.1f s, apply %.2f s (scaled)"
            % (time.perf_counter() - t0, o_fac, o_app))
        cpu = {"value": (per_matvec + o_app) * max(n_it), "unit": "s", "cores": threads, "kind": "oracle",
               "cpu_model": model, "cores_available": avail,
               "factor_s": o_fac, "factor_gflops": st["flops"] / o_fac / 1e9 if o_fac > 0 else None,
               "matvec_s": per_matvec, "apply_s": o_app, "rs_levels": o_detail,
               "sample": "PCG time = %d iterations x (one matvec + one apply).  Matvec: the oracle's dense FP64 "
                         "product (plain C, OpenMP, %d threads) on %d of %d rows x %d RHS (%.2f s), scaled by "
                         "N/rows (%.1f s).  Apply and factor: the oracle's RS steps (numpy/scipy) on %s boxes "
                         "per level of subdomain 0, scaled by each level's box count over all subdomains, plus "
                         "the roots' Cholesky and solve (apply %.2f s, factor %.1f s)"
                         % (max(n_it), threads, args.cpu_rows, N, nrhs, t_rows, per_matvec, "4", o_app, o_fac)}

    out = {
        "metric": METRIC,
        "value": pcg_s,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_total / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if prec == cbd.PREC_FP32 else "f64",
        "dtype_detail": ("f64: matvec, PCG recurrences, ID; f32: RS elimination, factor storage, apply"
                         if prec == cbd.PREC_FP32 else "f64 throughout"),
        "data": "synthetic",
        "config": {"workload": W["label"], "name": args.workload, "nrhs": nrhs, "n": n, "d": d,
                   "gpus": 1, "id_method": "gram" if idm == cbd.ID_GRAM else "qr"},
        "factor_s": factor_s,
        "factor_gflops": st["flops"] / factor_s / 1e9,
        "factor_flops": st["flops"],
        "S_last_level": st["S"],
        "factor_bytes": st["bytes"],
        "factor_launches": sched["launches"],
        "factor_host_syncs": 1 if box["replay"] else sched["host_syncs"],
        "factor_launch_mode": {"timed": "graph" if box["replay"] else "eager", "eager_s": fac_modes["eager"],
                               "graph_s": fac_modes["graph"], "eager_host_syncs": sched["host_syncs"],
                               "note": "graph: the factorization captured after an eager run (rs_factor_capture) "
                                       "and replayed every step (rs_factor_replay): every kernel runs again on the "
                                       "data, each value the eager run read back is checked on the device, one "
                                       "synchronization; eager: host planning between levels and a "
                                       "synchronization per read"},
        "n_it": [min(n_it), max(n_it)],
        "max_relres": max(rr_all),
        "pcg_launch_mode": {"timed": "graph" if box["graph"] else "eager", "eager_s": pcg_modes["eager"],
                            "graph_s": pcg_modes["graph"]},
        "matvec_avg_ms": mv_avg_s * 1e3 if mv_avg_s else None,
        "matvec_1rhs_ms": mv1_ms,
        "apply_avg_ms": ap_ms / max(ap_n, 1),
        "apply_tile": {"cols_per_level": box["apply_cols"], "chosen_by": "cbd_autotune_apply"},
        "matvec_tile": {"shape": tile, "rows_per_wave": 16 * (tile & 7), "waves_per_workgroup": 8 if tile >= 8 else 4,
                        "chosen_by": "cbd_autotune_matvec"},
        "sketched_id_variant": sketched,
        "other_id_method": alt_id,
        "bf16_gemm_variant": bf16,
        "pcg_with_fft_matvec": {"pcg_s": pcg_fft_s, "n_it": [min(its_fft), max(its_fft)],
                                "max_relres": max(rr_fft),
                                "note": "same factors; products with A by circulant-embedding FFT (Section 5 of "
                                        "the paper) instead of the dense on-the-fly matvec"} if full else None,
        "rank_predictor": {"train_s": mlp_train_s, "mean_abs_rank_err": sched["mean_abs_err"],
                           "held_out": mlp_held, "sketch_3d": mlp_gain_3d,
                           "factor_s_with": fac_modes["eager"], "factor_s_without": factor_nm_s,
                           "host_syncs_with": sched["host_syncs"], "host_syncs_without": sched_nm["host_syncs"],
                           "mispredicted_boxes": sched["mispredicted"]},
        "fp64_form": {"factor_s": f64_factor, "pcg_s_est": f64_pcg, "cols_timed": ncols,
                      "n_it": its64, "estimate": True,
                      "note": "PCG time measured on %d columns solved one at a time, scaled to %d"
                              % (ncols, nrhs)} if full else None,
        "fp64_factors_batched": f64_batched,
        "speedup_mixed_vs_fp64": {
            "total": (f64_pcg + f64_factor) / (pcg_s + factor_s),
            "pcg": f64_pcg / pcg_s, "factor": f64_factor / factor_s,
            "precision_pcg": f64_batched["pcg_s"] / pcg_s,
            "batching_pcg": f64_pcg / f64_batched["pcg_s"],
            "note": "precision_pcg: FP64 vs FP32 factors, both on all right-hand sides at once; "
                    "batching_pcg: FP64 factors one column at a time (estimated from the timed "
                    "columns) vs all at once"} if full else None,
        "u_err_vs_fp64_oracle": u_err or None,
        "u_err_note": ("column 0 of each form against the stored FP64 oracle solution "
                       "(oracle RS-PCG to 1e-12, tests/golden/u_512sq_cbd_col0.npy)") if u_err else None,
        "roofline": {"kernel": "kernel_matvec (FP64, %d RHS)" % nrhs, "bound": "mfma",
                     "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": measured_traffic(tile) if args.workload == "512sq" else None,
                     "library_dgemm_tflops": dgemm_ref,
                     "work": "2 N^2 nrhs FP64 flops per launch on FP64 MFMA (the N^2 kernel "
                             "evaluations run on the VALU and are not counted)"} if achieved else None,
        "factor_roofline": {"kernel": "rs_factor_batched (whole factorization)", "bound": "fp64",
                            "achieved": st["flops"] / factor_s / 1e12, "peak": FP64_PEAK_TFLOPS,
                            "unit": "TFLOP/s", "frac": st["flops"] / factor_s / 1e12 / FP64_PEAK_TFLOPS,
                            "work": "per-box flop formulas of the ID (FP64; the truncated pivoted QR's "
                                    "count, whichever route computes it), elimination and root "
                                    "Cholesky over the factor wall time; the ID runs in FP64, so the "
                                    "FP64 peak is the bound (FP32 peak for the elimination alone is "
                                    "157.3)"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""MI355X (gfx950) coloring-based overlapping domain-decomposition preconditioner
with recursive-skeletonization subdomain solvers (Chen & Biros, arXiv 2108.12574).

Thin Python binding of libcbd.so (C ABI in include/cbd.h).  Every step of the
method runs in the library's HIP kernels; this module only marshals arguments.
PyTorch provides device memory (FP64 CUDA tensors of shape (nrhs, N), i.e.
N x nrhs column-major) and the current stream.
"""
import ctypes

import torch

from . import _lib
from ._lib import (GRID_CELL, GRID_NODE, MODE_CBD, MODE_JACOBI, MODE_SCHWARZ, PREC_BF16GEMM,
                   PREC_FP32, PREC_FP64, ROWS_ALWAYS, ROWS_AUTO, ROWS_NEVER, ID_QR, ID_GRAM, CbdError, check,
                   lib)

__all__ = ["Problem", "Partition", "Factor", "RankMLP", "pcg_solve", "pcg_workspace", "timing", "CbdError",
           "GRID_CELL", "GRID_NODE", "MODE_JACOBI", "MODE_SCHWARZ", "MODE_CBD",
           "PREC_FP64", "PREC_FP32", "PREC_BF16GEMM", "ROWS_AUTO", "ROWS_NEVER", "ROWS_ALWAYS", "ID_QR", "ID_GRAM"]


def _free(fn, obj):
    """Release a library handle (quietly at interpreter shutdown)."""
    h = getattr(obj, "handle", None)
    L = getattr(_lib, "_lib", None) if _lib is not None else None
    if h and L is not None:
        try:
            getattr(L, fn)(h)
        except Exception:
            pass
    obj.handle = None


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _vec(x, N, device):
    """Check/normalize a (N,) or (nrhs, N) FP64 device tensor."""
    if x.dim() == 1:
        x = x.unsqueeze(0)
    if x.dtype != torch.float64 or x.device != device or x.shape[1] != N:
        raise ValueError("expected float64 tensor of shape (nrhs, %d) on %s" % (N, device))
    return x.contiguous()


class Problem:
    """Discretized IE (ie_assemble): A_ij = b_i h^d K(x_i - x_j) c_j, closed-form diagonal."""

    def __init__(self, d, n, grid=GRID_CELL, b=None, c=None, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.d, self.n, self.grid = d, n, grid
        self.N = n ** d
        f64 = dict(dtype=torch.float64, device=self.device)
        self.pts = torch.empty(d * self.N, **f64)
        self.diag = torch.empty(self.N, **f64)
        self.w = torch.empty(self.N, **f64)
        self.rowscale = torch.empty(self.N, **f64)
        self._b = None if b is None else torch.as_tensor(b, **f64).contiguous()
        self._c = None if c is None else torch.as_tensor(c, **f64).contiguous()
        h = ctypes.c_void_p()
        check(lib().ie_assemble(d, n, grid, _ptr(self._b), _ptr(self._c), _ptr(self.pts),
                                _ptr(self.diag), _ptr(self.w), _ptr(self.rowscale),
                                _stream(self.device), ctypes.byref(h)))
        self.handle = h

    def matvec(self, x):
        """y = A x for x of shape (N,) or (nrhs, N) (kernel_matvec)."""
        one = x.dim() == 1
        x = _vec(x, self.N, self.device)
        y = torch.empty_like(x)
        check(lib().kernel_matvec(self.handle, x.shape[0], _ptr(x), _ptr(y), _stream(self.device)))
        return y[0] if one else y

    def fft_prepare(self, max_pairs=8):
        """Set up the FFT matvec (cbd_fft_prepare) in a workspace this object keeps."""
        nb = lib().cbd_fft_workspace_bytes(self.d, self.n, max_pairs)
        ws = torch.empty(nb, dtype=torch.uint8, device=self.device)
        check(lib().cbd_fft_prepare(self.handle, max_pairs, _ptr(ws), nb, _stream(self.device)))
        self._fft_ws = ws

    def matvec_fft(self, x):
        """y = A x by FFT (kernel_matvec_fft); needs fft_prepare()."""
        one = x.dim() == 1
        x = _vec(x, self.N, self.device)
        y = torch.empty_like(x)
        check(lib().kernel_matvec_fft(self.handle, x.shape[0], _ptr(x), _ptr(y), _stream(self.device)))
        return y[0] if one else y

    def autotune_matvec(self, nrhs):
        """Pick the matvec tile shape for nrhs right-hand sides (cbd_autotune_matvec)."""
        ch = ctypes.c_int()
        cols = min(nrhs, 64)
        x = torch.empty(cols, self.N, dtype=torch.float64, device=self.device)
        y = torch.empty_like(x)
        check(lib().cbd_autotune_matvec(self.handle, nrhs, _ptr(x), _ptr(y), _stream(self.device),
                                        ctypes.byref(ch)))
        torch.cuda.synchronize(self.device)
        return ch.value

    def set_matvec_shape(self, nrhs, shape):
        """Fix the matvec tile shape for nrhs right-hand sides (cbd_matvec_set_shape)."""
        check(lib().cbd_matvec_set_shape(self.handle, nrhs, shape))

    def __del__(self, _free=_free):   # bound now: module globals are gone at shutdown
        _free("cbd_problem_free", self)


class Partition:
    """Domain decomposition and RS box hierarchy (dd_partition); host only.

    `grid` is a Problem, or a (d, n) pair (no GPU needed then).
    """

    def __init__(self, grid, m, delta=1, mode=MODE_CBD, leaf_side=0):
        d, n = (grid.d, grid.n) if isinstance(grid, Problem) else grid
        self.d, self.n = d, n
        h = ctypes.c_void_p()
        check(lib().dd_partition(d, n, m, delta, mode, leaf_side, ctypes.byref(h)))
        self.handle = h
        D, Lt, Lr, tot = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_long()
        check(lib().dd_partition_info(h, ctypes.byref(D), ctypes.byref(Lt), ctypes.byref(Lr),
                                      ctypes.byref(tot)))
        self.D, self.Lt, self.Lr, self.total = D.value, Lt.value, Lr.value, tot.value

    def subdomain(self, i):
        """(index list, number of leaves, root level) of subdomain i."""
        size, nl, rl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        check(lib().dd_subdomain_info(self.handle, i, ctypes.byref(size), ctypes.byref(nl),
                                      ctypes.byref(rl)))
        idx = (ctypes.c_int * size.value)()
        check(lib().dd_subdomain_index(self.handle, i, idx))
        return list(idx), nl.value, rl.value

    def level_boxes(self, i, level):
        """(lo/hi bounds, parent index) of the boxes of subdomain i at a level."""
        nb = ctypes.c_int()
        check(lib().dd_level_boxes(self.handle, i, level, ctypes.byref(nb), None, None))
        d = self.d
        lohi = (ctypes.c_int * (2 * d * nb.value))()
        par = (ctypes.c_int * nb.value)()
        check(lib().dd_level_boxes(self.handle, i, level, ctypes.byref(nb), lohi, par))
        boxes = [(list(lohi[b * 2 * d:b * 2 * d + d]), list(lohi[b * 2 * d + d:(b + 1) * 2 * d]))
                 for b in range(nb.value)]
        return boxes, list(par)

    def __del__(self, _free=_free):   # bound now: module globals are gone at shutdown
        _free("cbd_partition_free", self)


class Factor:
    """RS factors of all subdomain matrices (rs_factor_batched) and T^{-1} (rs_apply).

    The factor lives in a device workspace this object owns (a uint8 tensor, or `ws`
    if given), sized by rs_factor_workspace from `rank_hint` (ranks of an earlier
    factorization of the same layout, e.g. another Factor's `ranks`); if the ranks
    outgrow it, the library reports the bytes it needed and the call is repeated
    with more (up to three times).  `ranks` (device int32) holds every compressed box's
    rank in rs_factor_rank_count order."""

    def __init__(self, problem, partition, tol=1e-6, n_pxy=64, proxy_ratio=1.5,
                 precision=PREC_FP64, exact=False, mlp=None, row_compression=ROWS_AUTO, sketch_seed=None,
                 workspace_bytes=0, apply_rhs=64, rank_hint=None, ws=None, id_method=ID_QR, record=False):
        self.problem, self.partition = problem, partition
        self.precision = precision
        opts = _lib.RSOpts(tol, n_pxy, proxy_ratio, precision, 1 if exact else 0,
                           mlp.params.data_ptr() if mlp is not None else None, row_compression,
                           0 if sketch_seed is None else 1, 0 if sketch_seed is None else int(sketch_seed),
                           int(workspace_bytes), int(apply_rhs), int(id_method), 1 if record else 0)
        self.opts = opts
        self._mlp = mlp   # its parameters must outlive a captured graph
        cnt = ctypes.c_int()
        check(lib().rs_factor_rank_count(partition.handle, ctypes.byref(opts), ctypes.byref(cnt)))
        self.n_ranks = cnt.value
        hint = None
        if rank_hint is not None:
            import numpy as np
            hint = np.ascontiguousarray(torch.as_tensor(rank_hint).cpu().numpy(), dtype=np.int32)
            if hint.size != self.n_ranks:
                raise ValueError("rank_hint needs %d entries" % self.n_ranks)
        hp = hint.ctypes.data_as(ctypes.c_void_p) if hint is not None else None
        self.ranks = torch.zeros(max(self.n_ranks, 1), dtype=torch.int32, device=problem.device)
        if ws is None:
            nb = ctypes.c_size_t()
            check(lib().rs_factor_workspace(problem.handle, partition.handle, ctypes.byref(opts), hp,
                                            ctypes.byref(nb)))
            # an estimate above the free device memory is cut to it: levels then run in chunks
            free = torch.cuda.mem_get_info(problem.device)[0]
            ws = torch.empty(int(min(nb.value, 0.9 * free)), dtype=torch.uint8, device=problem.device)
        for attempt in range(4):
            h, used = ctypes.c_void_p(), ctypes.c_size_t()
            rc = lib().rs_factor_batched(problem.handle, partition.handle, ctypes.byref(opts), hp, _ptr(ws),
                                         ws.numel(), _ptr(self.ranks), ctypes.byref(used),
                                         _stream(problem.device), ctypes.byref(h))
            if rc != _lib.EWORKSPACE or attempt == 3:
                break
            # ranks above the estimate: the library reports a lower bound of what it needs
            # (up to the level that did not fit); grow past it with room for later levels
            grow = int(max(used.value * 1.5, ws.numel() * 2))
            del ws
            ws = torch.empty(grow, dtype=torch.uint8, device=problem.device)
        check(rc)
        self.handle = h
        self.ws = ws
        self.ws_used = used.value

    def capture(self):
        """Capture the factorization as a graph (rs_factor_capture; needs record=True).
        The graph workspace is a uint8 tensor this object keeps."""
        nb = lib().rs_factor_graph_bytes(self.handle)
        if nb == 0:
            raise ValueError("capture needs a Factor made with record=True")
        gws = torch.empty(nb, dtype=torch.uint8, device=self.problem.device)
        check(lib().rs_factor_capture(self.handle, _ptr(gws), nb, _stream(self.problem.device)))
        self._gws = gws

    @property
    def captured(self):
        """True once capture() has made a graph of this factorization."""
        return getattr(self, "_gws", None) is not None

    def replay(self):
        """Run the factorization again by replaying its graph (rs_factor_replay).  True
        when it reproduced the recording (the factor is valid for the problem's current
        data); False when it did not (the factor is stale: make a new Factor)."""
        rc = lib().rs_factor_replay(self.handle, _stream(self.problem.device))
        if rc == _lib.EREPLAN:
            return False
        check(rc)
        return True

    def apply(self, r):
        """z = T^{-1} r for r of shape (N,) or (nrhs, N)."""
        one = r.dim() == 1
        r = _vec(r, self.problem.N, self.problem.device)
        z = torch.empty_like(r)
        check(lib().rs_apply(self.handle, r.shape[0], _ptr(r), _ptr(z), _stream(self.problem.device)))
        return z[0] if one else z

    def autotune_apply(self, r):
        """Choose the apply sweep's shape level by level (cbd_autotune_apply) on a sample r
        of shape (nrhs, N); returns [(columns, threads)] per level ((0, 0): applied by GEMMs)."""
        r = _vec(r, self.problem.N, self.problem.device)
        n = self.stats()["levels"] + 1
        ch = (ctypes.c_int * (2 * n))()
        check(lib().cbd_autotune_apply(self.handle, r.shape[0], _ptr(r), _stream(self.problem.device), ch))
        return [(ch[2 * l], ch[2 * l + 1]) for l in range(n)]

    def set_apply_shapes(self, choices):
        """Fix the apply's shape per level (cbd_apply_set_shape): (columns, threads) pairs,
        e.g. the choices autotune_apply made on a factor of the same layout."""
        for l, (c, t) in enumerate(choices):
            check(lib().cbd_apply_set_shape(self.handle, l, int(c), int(t)))

    def apply_sub(self, i, r):
        """z = R_i^T A_i^{-1} R_i r, subdomain i's term of T^{-1} r (rs_apply_sub)."""
        one = r.dim() == 1
        r = _vec(r, self.problem.N, self.problem.device)
        z = torch.empty_like(r)
        check(lib().rs_apply_sub(self.handle, i, r.shape[0], _ptr(r), _ptr(z), _stream(self.problem.device)))
        return z[0] if one else z

    def stats(self):
        D = self.partition.D
        S = (ctypes.c_int * D)()
        nl, nb, fl = ctypes.c_int(), ctypes.c_size_t(), ctypes.c_double()
        check(lib().rs_factor_stats(self.handle, S, ctypes.byref(nl), ctypes.byref(nb), ctypes.byref(fl)))
        return {"S": list(S), "levels": nl.value, "bytes": nb.value, "flops": fl.value}

    def level(self, level):
        """(ranks, np, subdomain) per box of a batch level (level == levels: the roots)."""
        nb = ctypes.c_int()
        check(lib().rs_factor_level(self.handle, level, ctypes.byref(nb), None, None, None))
        k, npp, sub = ((ctypes.c_int * nb.value)() for _ in range(3))
        check(lib().rs_factor_level(self.handle, level, ctypes.byref(nb), k, npp, sub))
        return list(k), list(npp), list(sub)

    def box(self, i, level, b):
        """Host FP64 copy of one box factor: dict(sk, rd, T, E, Ginv, Bss)."""
        import numpy as np
        k, nr = ctypes.c_int(), ctypes.c_int()
        check(lib().rs_factor_box(self.handle, i, level, b, ctypes.byref(k), ctypes.byref(nr),
                                  None, None, None, None, None, None))
        k, nr = k.value, nr.value
        sk, rd = np.zeros(k, np.int32), np.zeros(nr, np.int32)
        T, E = np.zeros(k * nr), np.zeros(k * nr)
        Gi, Bss = np.zeros(nr * nr), np.zeros(k * k)
        ip = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        dp = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        kk, nn = ctypes.c_int(), ctypes.c_int()
        check(lib().rs_factor_box(self.handle, i, level, b, ctypes.byref(kk), ctypes.byref(nn),
                                  ip(sk), ip(rd), dp(T), dp(E), dp(Gi), dp(Bss)))
        f = lambda a, r, c: a.reshape(c, r).T   # column-major r x c
        return {"sk": sk, "rd": rd, "T": f(T, k, nr), "E": f(E, k, nr), "Ginv": f(Gi, nr, nr),
                "Bss": f(Bss, k, k)}

    def features(self, level):
        """Training pairs of one compressed level: (features (nbox, 6) float32, ranks (nbox,))."""
        import numpy as np
        nb = ctypes.c_int()
        check(lib().rs_factor_features(self.handle, level, ctypes.byref(nb), None, None))
        X = np.zeros((nb.value, RankMLP.F), np.float32)
        k = np.zeros(nb.value, np.int32)
        check(lib().rs_factor_features(self.handle, level, ctypes.byref(nb),
                                       X.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                       k.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return X, k

    def all_features(self):
        import numpy as np
        parts = [self.features(l) for l in range(self.stats()["levels"])]
        if not parts:
            return np.zeros((0, RankMLP.F), np.float32), np.zeros(0, np.int32)
        return np.concatenate([p[0] for p in parts]), np.concatenate([p[1] for p in parts])

    def schedule(self):
        """Stream synchronizations, stepped-QR launch pairs, mispredicted boxes, mean |k - k_pred|,
        row-compressed levels, sketch counts and level chunks of the factorization
        (rs_factor_schedule)."""
        v = [ctypes.c_int() for _ in range(10)]
        e = ctypes.c_double()
        nl = ctypes.c_long()
        check(lib().rs_factor_schedule(self.handle, ctypes.byref(v[0]), ctypes.byref(v[1]), ctypes.byref(v[2]),
                                       ctypes.byref(e), ctypes.byref(v[3]), ctypes.byref(v[4]), ctypes.byref(v[5]),
                                       ctypes.byref(v[6]), ctypes.byref(v[7]), ctypes.byref(v[8]), ctypes.byref(nl)))
        return {"host_syncs": v[0].value, "qr_steps": v[1].value, "mispredicted": v[2].value,
                "mean_abs_err": e.value, "row_compressed": v[3].value, "sketched": v[4].value,
                "sketch_fallbacks": v[5].value, "chunks": v[6].value, "sketched_pred": v[7].value,
                "sketch_pred_rejected": v[8].value, "launches": nl.value}

    def root(self, i):
        import numpy as np
        S = ctypes.c_int()
        check(lib().rs_factor_root(self.handle, i, ctypes.byref(S), None, None))
        idx = np.zeros(S.value, np.int32)
        Gi = np.zeros(S.value * S.value)
        check(lib().rs_factor_root(self.handle, i, ctypes.byref(S),
                                   idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                   Gi.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return idx, Gi.reshape(S.value, S.value).T

    def __del__(self, _free=_free):   # bound now: module globals are gone at shutdown
        _free("rs_factor_free", self)


class RankMLP:
    """Skeleton-rank predictor (rank_mlp_*): parameters on the device, trained by the
    library's forward/backward/Adam kernels on (features, log2(k + 1)) pairs."""

    F = 6

    def __init__(self, params, device="cuda"):
        self.device = torch.device(device)
        self.params = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        if self.params.numel() != lib().rank_mlp_params():
            raise ValueError("expected %d parameters" % lib().rank_mlp_params())
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    def _dev(self, a):
        return torch.as_tensor(a, dtype=torch.float32).to(self.device).contiguous()

    def forward(self, X):
        X = self._dev(X)
        y = torch.empty(X.shape[0], dtype=torch.float32, device=self.device)
        check(lib().rank_mlp_forward(_ptr(self.params), X.shape[0], _ptr(X), _ptr(y), _stream(self.device)))
        return y

    def loss_grad(self, X, t):
        X, t = self._dev(X), self._dev(t)
        n = X.shape[0]
        ws = torch.empty(lib().rank_mlp_workspace_bytes(n), dtype=torch.uint8, device=self.device)
        g = torch.empty_like(self.params)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        check(lib().rank_mlp_loss_grad(_ptr(self.params), n, _ptr(X), _ptr(t), _ptr(g), _ptr(loss), _ptr(ws),
                                       ws.numel(), _stream(self.device)))
        return loss, g

    def adam(self, g, lr):
        self.step += 1
        check(lib().rank_mlp_adam(_ptr(self.params), _ptr(g), _ptr(self.m), _ptr(self.v), self.step,
                                  ctypes.c_float(lr), _stream(self.device)))

    def train(self, X, k, steps=600, lr=1e-2):
        """Full-batch Adam on log2(k + 1); returns the final loss."""
        import math
        X = self._dev(X)
        t = self._dev(torch.log2(torch.as_tensor(k, dtype=torch.float32) + 1.0))
        loss = None
        for s in range(steps):
            loss, g = self.loss_grad(X, t)
            self.adam(g, lr * (0.5 * (1 + math.cos(math.pi * s / steps))) + 1e-4)
        return float(loss.item())

    def predict_ranks(self, X):
        y = self.forward(X)
        return torch.clamp(torch.round(torch.exp2(y) - 1.0), min=0).to(torch.int64)


def pcg_workspace(problem, nrhs):
    """A device workspace for pcg_solve with nrhs right-hand sides (pcg_workspace_bytes)."""
    return torch.empty(lib().pcg_workspace_bytes(problem.N, nrhs), dtype=torch.uint8, device=problem.device)


def pcg_solve(problem, factor, f, tol=1e-10, maxit=200, flexible=False, graph=False, fft=False, ws=None):
    """PCG on A u = f (pcg_solve).  f: (N,) or (nrhs, N).  Returns (u, iters, relres).

    graph=True replays each iteration from captured HIP graphs (needs a non-default
    current stream).  ws: a workspace from pcg_workspace (allocated here if None)."""
    one = f.dim() == 1
    f = _vec(f, problem.N, problem.device)
    nrhs = f.shape[0]
    u = torch.empty_like(f)
    nb = lib().pcg_workspace_bytes(problem.N, nrhs)
    if ws is None or ws.numel() < nb:
        ws = pcg_workspace(problem, nrhs)
    iters = (ctypes.c_int * nrhs)()
    relres = (ctypes.c_double * nrhs)()
    flags = (1 if flexible else 0) | (2 if graph else 0) | (4 if fft else 0)
    rc = lib().pcg_solve(problem.handle, factor.handle if factor is not None else None, nrhs,
                         _ptr(f), _ptr(u), tol, maxit, flags, _ptr(ws), nb,
                         iters, relres, _stream(problem.device))
    check(rc, allow_warning=True)
    its, rr = list(iters), list(relres)
    if one:
        return u[0], its[0], rr[0]
    return u, its, rr


class timing:
    """HIP-event timers the library records around its launches (per family)."""

    @staticmethod
    def enable(on=True):
        check(lib().cbd_timing_enable(1 if on else 0))

    @staticmethod
    def reset():
        check(lib().cbd_timing_reset())

    @staticmethod
    def get(name):
        ms, n = ctypes.c_double(), ctypes.c_long()
        check(lib().cbd_timing_get(name.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

"""ctypes loader of the oracle's plain C dense matvec (oracle/c/matvec.c).

Test infrastructure only.  The library is compiled with gcc on first use (or
by the package build step) into oracle/c/.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "c", "matvec.c")
_LIB = os.path.join(_HERE, "c", "libcbd_oracle.so")
_lib = None


def build(force=False):
    """Compile the oracle C library with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        lib.oracle_matvec.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, dp, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, dp, lp, ctypes.c_long, dp]
        lib.oracle_matvec.restype = None
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def matvec(prob, X, rows=None):
    """A_bc @ X for X of shape (N,) or (N, nrhs); only the given rows if rows is not None.

    prob: an oracle.ie.Problem.  Returns shape (nrows,) or (nrows, nrhs).
    """
    lib = _load()
    X = np.asarray(X, dtype=np.float64)
    one = X.ndim == 1
    Xr = np.ascontiguousarray(X[:, None] if one else X)
    nrhs = Xr.shape[1]
    pts = np.ascontiguousarray(prob.x, dtype=np.float64)
    b = np.ascontiguousarray(prob.b)
    c = np.ascontiguousarray(prob.c)
    if rows is None:
        nrows = prob.N
        rp = None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        nrows = len(rows)
        rp = rows.ctypes.data_as(ctypes.POINTER(ctypes.c_long))
    Y = np.zeros((nrows, nrhs))
    lib.oracle_matvec(prob.d, prob.N, _dp(pts), _dp(b), _dp(c), prob.weight, prob.a_self,
                      nrhs, _dp(Xr), rp, nrows, _dp(Y))
    return Y[:, 0] if one else Y

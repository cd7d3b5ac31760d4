"""Randomized (sketched) interpolative decomposition.

Test infrastructure only: this module is part of the CPU oracle and is never
imported by the GPU library.

The paper's last 3D experiments compute the IDs with a randomized scheme (after
Halko, Martinsson and Tropp, cited in its conclusions as the way around the ID
being the bottleneck).  The reading used here: the ID of the columns of Y
(m x n) is taken from the truncated CPQR of the sketch Z = Omega Y, with Omega
an ell x m matrix of independent random signs.  If Y = Y[:, s] T exactly with
k columns and ell > k, then Z = Z[:, s] T, so the ID of Z is an ID of Y; for
numerically low-rank Y the error stays near the tolerance with high
probability.  Readings (the paper gives no details):
* sketch size ell = ceil(3 n / 5) + 8; no sketch when ell >= min(m, n);
* the CPQR of Z uses the same rank and tie rules as the deterministic ID;
* a sketch whose rank k exceeds ell - 8 is taken as saturated (the sketch may
  have missed part of the range): the box falls back to the deterministic ID;
* with a predicted rank k_p of the box (from the rank predictor, or the ranks of
  an earlier factorization), a first sketch of ell_p = 4 k_p + 32 rows is tried
  when that is below the shape-based size; its ID is kept if k <= ell_p / 4 (an
  oversampling of four, after Halko, Martinsson and Tropp's analysis of the
  range finder), else the box goes on to the shape-based sketch.  The first
  ell_p rows of Omega are the same in both (the signs depend on the row index);
* the signs are a counter-based hash, so that any implementation can draw the
  same Omega: sign(seed, box key, i, row key) is the top bit of the splitmix64
  output function (Steele, Lea and Flood, OOPSLA 2014) applied to
  seed + key * G1 + i * G2 + rowkey * G3 (mod 2^64), + for 0 and - for 1, with
  G1 = 0x9E3779B97F4A7C15, G2 = 0xD1B54A32D192ED03, G3 = 0x8CB92BA72F3D8DD7.
  The row key of a near-field row is the global index of its point; of proxy
  row q it is N + q; the box key is (subdomain << 40) | (level << 32) | box.
"""
import numpy as np

from .cpqr import interp_decomp, TIE_FP64

M64 = (1 << 64) - 1
G1, G2, G3 = 0x9E3779B97F4A7C15, 0xD1B54A32D192ED03, 0x8CB92BA72F3D8DD7
OVER = 8


def mix64(x):
    """The splitmix64 output function on uint64 array(s) (arithmetic mod 2^64)."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def box_key(sub, level, box):
    return (int(sub) << 40) | (int(level) << 32) | int(box)


def signs(seed, key, ell, rowkeys):
    """Omega (ell x len(rowkeys)) of +-1 for one box."""
    i = np.arange(ell, dtype=np.uint64)[:, None]
    r = np.asarray(rowkeys, dtype=np.uint64)[None, :]
    base = np.uint64((int(seed) + int(key) * G1) & M64)
    with np.errstate(over="ignore"):
        x = base + i * np.uint64(G2) + r * np.uint64(G3)
    top = mix64(x) >> np.uint64(63)
    return 1.0 - 2.0 * top.astype(np.float64)


def sketch_size(m, n):
    """ell for an m x n matrix, or 0 when the deterministic ID is used directly."""
    ell = (3 * n + 4) // 5 + OVER
    return ell if ell < min(m, n) else 0


PRED_FACTOR, PRED_EXTRA = 4, 32


def predicted_sketch_size(m, n, k_pred):
    """ell from a predicted rank, or 0 when it would not be below the shape-based size."""
    ell_shape = sketch_size(m, n)
    ell = PRED_FACTOR * max(int(k_pred), 0) + PRED_EXTRA
    return ell if ell_shape and ell < ell_shape else 0


def interp_decomp_sketched(Y, tol, seed, key, rowkeys, tie=TIE_FP64, k_pred=None):
    """ID of the columns of Y from the CPQR of Omega Y.  Returns (k, perm, T, how) with how
    0 (deterministic ID), 1 (shape-based sketch) or 2 (rank-sized sketch).
    k_pred: a predicted rank of the box, or None."""
    m, n = Y.shape
    if k_pred is not None:
        ell = predicted_sketch_size(m, n, k_pred)
        if ell:
            Z = signs(seed, key, ell, rowkeys) @ Y
            k, perm, T = interp_decomp(Z, tol, tie)
            if PRED_FACTOR * k <= ell:
                return k, perm, T, 2
    ell = sketch_size(m, n)
    if ell:
        Z = signs(seed, key, ell, rowkeys) @ Y
        k, perm, T = interp_decomp(Z, tol, tie)
        if k <= ell - OVER:
            return k, perm, T, 1
    k, perm, T = interp_decomp(Y, tol, tie)
    return k, perm, T, 0

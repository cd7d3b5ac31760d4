"""Preconditioned conjugate gradients (Section 5, PCG on (e:axb)).

Per right-hand side, independently: x0 = 0, r0 = f, z0 = M r0, p0 = z0;
alpha = r.z / p.Ap; x += alpha p; r -= alpha Ap; stop when ||r||_2/||f||_2 <= tol;
beta = r+.z+ / r.z (or the flexible Polak-Ribiere form r+.(z+ - z) / r.z);
p = z + beta p.  The iteration count is the number of products with A.
"""
import numpy as np


def pcg(matvec, precond, f, tol=1e-10, maxit=200, flexible=False):
    """Solve A u = f column by column.  f: (N,) or (N, nrhs).  Returns (u, iters, relres).

    matvec(X) and precond(X) take and return (N, k) arrays; a column that has
    converged is frozen.
    """
    f = np.asarray(f, dtype=np.float64)
    one = f.ndim == 1
    F = f[:, None] if one else f
    N, nrhs = F.shape
    u = np.zeros_like(F)
    r = F.copy()
    fn = np.sqrt(np.sum(F * F, axis=0))
    iters = np.zeros(nrhs, dtype=np.int64)
    relres = np.ones(nrhs)
    done = fn == 0.0
    relres[done] = 0.0
    z = precond(r) if precond is not None else r.copy()
    p = z.copy()
    rz = np.sum(r * z, axis=0)
    for it in range(1, maxit + 1):
        act = np.nonzero(~done)[0]
        if len(act) == 0:
            break
        q = matvec(p[:, act])
        alpha = rz[act] / np.sum(p[:, act] * q, axis=0)
        u[:, act] += alpha * p[:, act]
        r[:, act] -= alpha * q
        iters[act] = it
        rel = np.sqrt(np.sum(r[:, act] ** 2, axis=0)) / fn[act]
        relres[act] = rel
        conv = rel <= tol
        done[act[conv]] = True
        act = act[~conv]
        if len(act) == 0:
            break
        znew = precond(r[:, act]) if precond is not None else r[:, act].copy()
        rznew = np.sum(r[:, act] * znew, axis=0)
        if flexible:
            beta = np.sum(r[:, act] * (znew - z[:, act]), axis=0) / rz[act]
        else:
            beta = rznew / rz[act]
        p[:, act] = znew + beta * p[:, act]
        z[:, act] = znew
        rz[act] = rznew
    if one:
        return u[:, 0], int(iters[0]), float(relres[0])
    return u, iters, relres

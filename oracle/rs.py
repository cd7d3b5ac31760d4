"""Recursive skeletonization (RS) of every subdomain matrix A_i, and its apply.

Section 4.2 of the paper.  For each subdomain (subproblem A_i = R_i A R_i^T,
(e:ai)), level by level over the box hierarchy of oracle.dd:

1. for every box p at the level: compress its off-diagonal block with an ID
   (e:id), using the proxy trick: the far field is replaced by the active DOFs
   of other boxes inside a proxy circle/sphere plus kernel rows from points on
   that surface (radius proxy_ratio x box side);
2. compress-then-eliminate (e:al), (e:alu), (e:b):
     B_rr = A_rr - A_rs T - T^T A_sr + T^T A_ss T,  B_sr = A_sr - A_ss T,
     B_rr = G^T G (Cholesky),  E = B_sr G^{-1},  B_ss = A_ss - E E^T;
3. the next level's box matrix is the Schur complement (e:schur) restricted to
   the box: children's B_ss on the diagonal, original entries of A between
   different children;
4. one box left: Cholesky of the last Schur complement.

All boxes of a level are compressed against the DOFs active at the start of
the level (level-parallel reading).  The paper proceeds box by box: once a box
is eliminated, its redundant DOFs leave the active set, so a later box of the
same level sees only the earlier boxes' skeletons in its near field (the
off-diagonal blocks between boxes are unchanged by an elimination, (e:schur)).
order="sequential" takes that reading, in the level's box order; the
level-parallel near fields are supersets of those rows.

The apply (the inverse of the factorization, used for T^{-1} of (e:ad)):
forward over levels  v_r -= T^T v_s; v_r = G^{-T} v_r; v_s -= E v_r,
root solve, backward  v_r -= E^T v_s; v_r = G^{-1} v_r; v_s -= T v_r.

Parity: skeleton sets are pinned only indirectly (ID error against the full far
field, apply error against exact subdomain solves, PCG solution against dense
Cholesky); the choice of skeletons has several correct answers.
"""
import numpy as np
from scipy.linalg import cholesky, solve_triangular, cho_solve

from . import ie
from .cpqr import interp_decomp, TIE_FP64
from . import sketch


class NotSPDError(RuntimeError):
    pass


def proxy_directions(d, n_pxy):
    """Unit vectors of the proxy surface: n_pxy equispaced angles on the circle (2D);
    a Fibonacci (golden-angle) point set on the sphere (3D)."""
    j = np.arange(n_pxy, dtype=np.float64)
    if d == 2:
        th = 2.0 * np.pi * j / n_pxy
        return np.stack([np.cos(th), np.sin(th)], axis=1)
    z = 1.0 - (2.0 * j + 1.0) / n_pxy
    rr = np.sqrt(1.0 - z * z)
    phi = j * (np.pi * (3.0 - np.sqrt(5.0)))
    return np.stack([rr * np.cos(phi), rr * np.sin(phi), z], axis=1)


def _grid_coords(g, n, d):
    out = []
    for _ in range(d):
        out.append(g % n)
        g = g // n
    return np.stack(out, axis=1)


class BoxFactor:
    def __init__(self, sk, rd, T, G, E, Bss):
        self.sk, self.rd, self.T, self.G, self.E, self.Bss = sk, rd, T, G, E, Bss


class SubdomainFactor:
    def __init__(self):
        self.levels = []       # levels[l] = list of BoxFactor (box order of that level)
        self.root = None       # local indices of the root DOFs
        self.root_G = None     # upper Cholesky factor of the last Schur complement
        self.root_A = None
        self.sketched = 0      # boxes whose ID came from a sketch
        self.sketched_pred = 0 # of those, from the rank-sized first sketch


def proxy_matrix(prob, sd, box, p, cand, n_pxy=64, proxy_ratio=1.5):
    """The matrix whose ID compresses box `box` of subdomain sd (step 1 above):
    rows A(near, p) for the candidates `cand` (subdomain-local indices of other
    boxes' active DOFs) strictly inside the proxy surface, tested exactly in
    half-cell units, |2j+1-(lo+hi)|^2 < (2 ratio L)^2; then the kernel from the
    proxy points ctr + rho dir_q to the box's points, scaled by the column weights.
    Returns (Y, near)."""
    d, n, h = prob.d, prob.n, prob.h
    gidx = sd.index
    lo, hi = np.array(box.lo), np.array(box.hi)
    L = int(np.max(hi - lo))
    cand = np.asarray(cand, dtype=np.int64)
    off = 2 * _grid_coords(gidx[cand], n, d) + 1 - (lo + hi)[None, :]
    near = cand[np.sum(off * off, axis=1) < (2.0 * proxy_ratio * L) ** 2]
    ctr = 0.5 * (lo + hi) * h
    rho = proxy_ratio * L * h
    pxy = ctr[None, :] + rho * proxy_directions(d, n_pxy)
    Yn = prob.block(gidx[near], gidx[p])
    diff = pxy[:, None, :] - prob.x[gidx[p]][None, :, :]
    w = prob.weight * prob.c[gidx[p]]          # column scale of a proxy row
    Yp = ie.kernel(d, np.sqrt(np.sum(diff * diff, axis=2))) * w[None, :]
    return np.vstack([Yn, Yp]), near


def eliminate_box(App, ps, pr, T):
    """Compress-then-eliminate one box (step 2 above): App its box matrix, ps / pr the
    positions of its skeleton / redundant DOFs in App, T its ID coefficients.
    Returns (G, E, B_ss); raises NotSPDError if B_rr is not positive definite."""
    Ass = App[np.ix_(ps, ps)]
    Asr = App[np.ix_(ps, pr)]
    Ars = App[np.ix_(pr, ps)]
    Arr = App[np.ix_(pr, pr)]
    # (e:al)
    Brr = Arr - Ars @ T - T.T @ Asr + T.T @ Ass @ T
    Bsr = Asr - Ass @ T
    if len(pr) == 0:
        return np.zeros((0, 0)), np.zeros((len(ps), 0)), Ass.copy()
    Brr = 0.5 * (Brr + Brr.T)
    try:
        G = cholesky(Brr, lower=False)
    except np.linalg.LinAlgError:
        raise NotSPDError("B_rr not SPD")
    # (e:alu)/(e:b): E = B_sr G^{-1}, B_ss = A_ss - E E^T
    E = solve_triangular(G, Bsr.T, trans="T", lower=False).T
    return G, E, Ass - E @ E.T


def box_forward(b, v):
    """The forward sweep's step for box b (a BoxFactor) on v (rows: the DOFs b.sk, b.rd index)."""
    if len(b.rd) == 0:
        return
    vr = v[b.rd] - b.T.T @ v[b.sk]
    vr = solve_triangular(b.G, vr, trans="T", lower=False)
    v[b.sk] -= b.E @ vr
    v[b.rd] = vr


def box_backward(b, v):
    """The backward sweep's step for box b on v."""
    if len(b.rd) == 0:
        return
    vr = v[b.rd] - b.E.T @ v[b.sk]
    vr = solve_triangular(b.G, vr, lower=False)
    v[b.sk] -= b.T @ vr
    v[b.rd] = vr


def factor_subdomain(prob, part, sd, tol, n_pxy=64, proxy_ratio=1.5, tie=TIE_FP64,
                     keep_matrices=False, sketch_seed=None, sub=0, order="level", rank_pred=None):
    """RS factorization of A_i for one subdomain (Section 4.2).  With sketch_seed set,
    every ID is the randomized one of oracle.sketch (subdomain index `sub` enters
    the box keys of the random signs).  order: "level" (near fields from the DOFs
    active at the start of the level) or "sequential" (box by box: the redundant
    DOFs of boxes already eliminated at this level are no longer active).  rank_pred:
    {(level, box): predicted rank} for the first, rank-sized sketch of oracle.sketch."""
    if order not in ("level", "sequential"):
        raise ValueError("order must be 'level' or 'sequential'")
    if prob.grid != ie.GRID_CELL:
        raise ValueError("RS is defined on the cell-centred grid")
    gidx = sd.index
    n_dirs = len(proxy_directions(prob.d, n_pxy))
    f = SubdomainFactor()
    # level 0: each leaf box holds its points; its matrix is A(p, p)
    active = [np.arange(st, st + cnt) for (_, _, st, cnt) in sd.leaves]
    boxmat = [prob.block(gidx[a], gidx[a]) for a in active]
    for l in range(sd.root_level):
        boxes = sd.levels[l]
        owner = np.concatenate([np.full(len(a), bi) for bi, a in enumerate(active)])
        allact = np.concatenate(active)
        alive = np.ones(len(allact), dtype=bool)      # still active (sequential order)
        lvl = []
        for bi, box in enumerate(boxes):
            p = active[bi]
            # near field: other boxes' active DOFs strictly inside the proxy surface
            Y, near = proxy_matrix(prob, sd, box, p, allact[(owner != bi) & alive], n_pxy, proxy_ratio)
            if sketch_seed is None:
                k, perm, T = interp_decomp(Y, tol, tie)
            else:
                rowkeys = np.concatenate([gidx[near], prob.N + np.arange(n_dirs)])
                k_pred = None if rank_pred is None else rank_pred.get((l, bi))
                k, perm, T, used = sketch.interp_decomp_sketched(
                    Y, tol, sketch_seed, sketch.box_key(sub, l, bi), rowkeys, tie, k_pred=k_pred)
                f.sketched += int(used > 0)
                f.sketched_pred += int(used == 2)
            ps, pr = perm[:k], perm[k:]
            try:
                G, E, Bss = eliminate_box(boxmat[bi], ps, pr, T)
            except NotSPDError:
                raise NotSPDError(f"B_rr not SPD at level {l} box {bi}")
            lvl.append(BoxFactor(p[ps], p[pr], T, G, E, Bss))
            if order == "sequential":
                alive[np.isin(allact, p[pr])] = False
        f.levels.append(lvl)
        # next level: union of children's skeletons; matrix per (e:schur)
        new_active, new_mat = [], []
        for pbox in sd.levels[l + 1]:
            ch = pbox.children
            sks = [lvl[c].sk for c in ch]
            act = np.concatenate(sks)
            mat = np.zeros((len(act), len(act)))
            offs = np.cumsum([0] + [len(s) for s in sks])
            for a, ca in enumerate(ch):
                for b, cb in enumerate(ch):
                    blk = (slice(offs[a], offs[a + 1]), slice(offs[b], offs[b + 1]))
                    if a == b:
                        mat[blk] = lvl[ca].Bss
                    elif len(sks[a]) and len(sks[b]):
                        mat[blk] = prob.block(gidx[sks[a]], gidx[sks[b]])
            new_active.append(act)
            new_mat.append(mat)
        active, boxmat = new_active, new_mat
    # last level: Cholesky of the remaining Schur complement
    f.root = active[0]
    S = 0.5 * (boxmat[0] + boxmat[0].T)
    try:
        f.root_G = cholesky(S, lower=False) if len(f.root) else np.zeros((0, 0))
    except np.linalg.LinAlgError:
        raise NotSPDError("root Schur complement not SPD")
    if keep_matrices:
        f.root_A = S
    return f


class RSPreconditioner:
    """T^{-1} = sum_i R_i^T A_i^{-1} R_i (e:ad) with A_i^{-1} applied through RS factors."""

    def __init__(self, prob, part, tol, n_pxy=64, proxy_ratio=1.5, tie=TIE_FP64, sketch_seed=None,
                 order="level", rank_pred=None):
        """rank_pred: {(subdomain, level, box): predicted rank} or None (sketched IDs only)."""
        self.prob, self.part = prob, part
        per_sub = lambda i: None if rank_pred is None else {(l, b): k for (j, l, b), k in rank_pred.items() if j == i}
        self.subs = [factor_subdomain(prob, part, sd, tol, n_pxy, proxy_ratio, tie,
                                      sketch_seed=sketch_seed, sub=i, order=order, rank_pred=per_sub(i))
                     for i, sd in enumerate(part.subdomains)]

    def apply_sub(self, i, v):
        """A_i^{-1} v approximately, v of shape (n_i, nrhs) in local numbering."""
        f = self.subs[i]
        v = np.array(v, dtype=np.float64, copy=True)
        for lvl in f.levels:
            for b in lvl:
                box_forward(b, v)
        if len(f.root):
            v[f.root] = cho_solve((f.root_G, False), v[f.root])
        for lvl in reversed(f.levels):
            for b in lvl:
                box_backward(b, v)
        return v

    def apply(self, r):
        """z = T^{-1} r for r of shape (N,) or (N, nrhs)."""
        r = np.asarray(r, dtype=np.float64)
        one = r.ndim == 1
        R = r[:, None] if one else r
        z = np.zeros_like(R)
        for i, sd in enumerate(self.part.subdomains):
            z[sd.index] += self.apply_sub(i, R[sd.index])
        return z[:, 0] if one else z

    def stats(self):
        """Per subdomain: DOFs at the last level S, and per-level rank lists."""
        out = []
        for f in self.subs:
            out.append({"S": len(f.root),
                        "ranks": [[len(b.sk) for b in lvl] for lvl in f.levels],
                        "np": [[len(b.sk) + len(b.rd) for b in lvl] for lvl in f.levels]})
        return out

"""Domain decompositions and the per-subdomain box hierarchy.

Sections 2.2-2.3 of the paper: uniform partition (e:dd), one-layer extension,
Schwarz subdomains (e:first), coloring-based subdomains (e:cbd)/(e:second),
block-Jacobi subdomains (table t:dd); and the hierarchical partitioning of a
subdomain used by recursive skeletonization (Section 4.2, around (e:oi) and
(e:schur): leaf regions, merged by spatial proximity until one box is left).

Readings (where the paper leaves a choice):
* extension by `delta` layers per side, clipped at the domain boundary;
* coloring c(k) = sum_t (k_t mod 2) 2^(t-1) (2^d colors, the theorem of Section 2.3);
* leaf boxes: each extended partition of a subdomain is a region; a region is one
  leaf box, or is tiled by `leaf_side`-wide tiles (ragged at its far edges);
* level l box key = (k' >> max(0, l - Lt), q >> min(l, Lt)), with k' = floor(k/2)
  (CBD) or 0, q the tile coordinate; Lt, Lr from the largest tile / region grid;
* boxes at a level are ordered by first appearance in leaf order; a subdomain's
  root is its first level with a single box.
"""
import numpy as np

JACOBI = 0
SCHWARZ = 1
CBD = 2


def _ceil_log2(v):
    l = 0
    while (1 << l) < v:
        l += 1
    return l


def _lin(q, ext):
    """Linear index of a multi-index q over extents ext, first axis fastest."""
    out, mul = 0, 1
    for qt, et in zip(q, ext):
        out += qt * mul
        mul *= et
    return out


def _unlin(i, ext):
    q = []
    for et in ext:
        q.append(i % et)
        i //= et
    return tuple(q)


def _grid_indices(d, n, lo, hi):
    """Global indices of the points in the cell box [lo, hi) in lexicographic order (x fastest)."""
    ranges = [np.arange(lo[t], hi[t], dtype=np.int64) for t in range(d)]
    mesh = np.meshgrid(*ranges, indexing="ij")
    g = np.zeros(mesh[0].shape, dtype=np.int64)
    mul = 1
    for t in range(d):
        g = g + mesh[t] * mul
        mul *= n
    return np.ascontiguousarray(g.transpose().reshape(-1))


class Box:
    """A box of the hierarchy: cell bounding box [lo, hi) and its members."""

    def __init__(self, key, lo, hi):
        self.key = key
        self.lo = list(lo)
        self.hi = list(hi)
        self.children = []      # indices into the previous level (level > 0)
        self.leaf = -1          # leaf index (level 0)


class Subdomain:
    """One subdomain Omega_i: global index list I_i in local order and its box levels."""

    def __init__(self):
        self.index = None       # int64 global indices, local numbering order
        self.leaves = []        # (lo, hi, local_start, count)
        self.levels = []        # levels[l] = list of Box
        self.root_level = 0


class Partition:
    """Domain decomposition of the n^d grid (Sections 2.2-2.3) plus RS box hierarchies.

    mode: JACOBI (Omega_i = P_i), SCHWARZ (Omega_i = extended P_i), CBD
    (Omega_i = union of same-color extended P_k).  leaf_side = 0 makes each
    extended partition one leaf box.
    """

    def __init__(self, d, n, m, delta=1, mode=CBD, leaf_side=0):
        if n % m != 0:
            raise ValueError("n must be a multiple of m")
        if mode == JACOBI:
            delta = 0
        s = n // m
        if mode == CBD and m > 2 and 2 * delta > s:
            raise ValueError("CBD needs 2*delta <= n/m so same-color regions are disjoint")
        self.d, self.n, self.m, self.delta, self.mode, self.leaf_side = d, n, m, delta, mode, leaf_side
        M = m ** d
        regions_of = []          # per subdomain: list of (kprime, lo, hi)
        if mode in (JACOBI, SCHWARZ):
            for kl in range(M):
                k = _unlin(kl, [m] * d)
                lo = [max(0, k[t] * s - delta) for t in range(d)]
                hi = [min(n, (k[t] + 1) * s + delta) for t in range(d)]
                regions_of.append([((0,) * d, lo, hi)])
        elif mode == CBD:
            regions_of = [[] for _ in range(2 ** d)]
            for kl in range(M):
                k = _unlin(kl, [m] * d)
                color = sum((k[t] % 2) << t for t in range(d))
                lo = [max(0, k[t] * s - delta) for t in range(d)]
                hi = [min(n, (k[t] + 1) * s + delta) for t in range(d)]
                regions_of[color].append((tuple(kt // 2 for kt in k), lo, hi))
        else:
            raise ValueError("unknown mode")
        # tiles per axis of every region, and the global level counts Lt, Lr
        def tiles_per_axis(lo, hi):
            if leaf_side <= 0:
                return [1] * d
            return [-(-(hi[t] - lo[t]) // leaf_side) for t in range(d)]
        qmax, rmax = 1, 1
        for regs in regions_of:
            for kp, lo, hi in regs:
                qmax = max(qmax, max(tiles_per_axis(lo, hi)))
                rmax = max(rmax, max(kp) + 1)
        self.Lt = _ceil_log2(qmax)
        self.Lr = _ceil_log2(rmax)
        self.subdomains = []
        for regs in regions_of:
            sd = Subdomain()
            leaf_keys = []       # (kprime, q) per leaf
            idx_parts = []
            start = 0
            for kp, lo, hi in regs:
                T = tiles_per_axis(lo, hi)
                for ql in range(int(np.prod(T))):
                    q = _unlin(ql, T)
                    if leaf_side <= 0:
                        tlo, thi = list(lo), list(hi)
                    else:
                        tlo = [lo[t] + q[t] * leaf_side for t in range(d)]
                        thi = [min(hi[t], lo[t] + (q[t] + 1) * leaf_side) for t in range(d)]
                    g = _grid_indices(d, n, tlo, thi)
                    sd.leaves.append((tlo, thi, start, len(g)))
                    leaf_keys.append((kp, q))
                    idx_parts.append(g)
                    start += len(g)
            sd.index = np.concatenate(idx_parts)
            # levels: a leaf's key at level l decides its box; boxes in order of first appearance
            l = 0
            leaf_box_prev = None
            while True:
                boxes, where, leaf_box = [], {}, []
                for li, (kp, q) in enumerate(leaf_keys):
                    key = (tuple(v >> max(0, l - self.Lt) for v in kp),
                           tuple(v >> min(l, self.Lt) for v in q))
                    lo, hi = sd.leaves[li][0], sd.leaves[li][1]
                    if key not in where:
                        where[key] = len(boxes)
                        boxes.append(Box(key, lo, hi))
                    b = boxes[where[key]]
                    b.lo = [min(b.lo[t], lo[t]) for t in range(d)]
                    b.hi = [max(b.hi[t], hi[t]) for t in range(d)]
                    if l == 0:
                        b.leaf = li
                    leaf_box.append(where[key])
                if l > 0:
                    # children of a box: previous-level boxes (in their order) whose leaves it holds
                    for c in range(len(sd.levels[l - 1])):
                        first_leaf = leaf_box_prev.index(c)
                        boxes[leaf_box[first_leaf]].children.append(c)
                sd.levels.append(boxes)
                leaf_box_prev = leaf_box
                if len(boxes) == 1:
                    sd.root_level = l
                    break
                l += 1
            self.subdomains.append(sd)

    @property
    def D(self):
        return len(self.subdomains)

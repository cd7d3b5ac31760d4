"""Pins of the oracle's decompositions (Sections 2.2-2.3) and box hierarchy (Section 4.2)."""
import numpy as np
import pytest

from oracle import dd


def test_extended_partition_sizes():
    # Section 2.2: interior extended partitions have (n/m + 2)^d points
    p = dd.Partition(2, 64, 16, 1, dd.SCHWARZ)
    sizes = sorted({len(sd.index) for sd in p.subdomains})
    assert sizes == [25, 30, 36]
    assert p.D == 256
    p3 = dd.Partition(3, 16, 4, 1, dd.SCHWARZ)
    assert max(len(sd.index) for sd in p3.subdomains) == 6 ** 3


def test_jacobi_is_a_partition():
    p = dd.Partition(2, 32, 4, 5, dd.JACOBI)   # delta ignored for Jacobi
    allidx = np.concatenate([sd.index for sd in p.subdomains])
    assert np.array_equal(np.sort(allidx), np.arange(32 * 32))


@pytest.mark.parametrize("d,n,m", [(2, 64, 16), (2, 32, 2), (3, 16, 4), (2, 60, 6)])
def test_cbd_colors_cover_and_are_disjoint_inside(d, n, m):
    p = dd.Partition(d, n, m, 1, dd.CBD)
    assert p.D == 2 ** d          # theorem of Section 2.3: 2^d colors
    allidx = np.concatenate([sd.index for sd in p.subdomains])
    assert np.array_equal(np.unique(allidx), np.arange(n ** d))
    for sd in p.subdomains:
        assert len(np.unique(sd.index)) == len(sd.index)


def test_cbd_same_color_regions_not_adjacent():
    # the coloring gives adjacent partitions (corners included) different colors
    m = 6
    for k1 in range(m):
        for k2 in range(m):
            c = (k1 % 2) + 2 * (k2 % 2)
            for a in (-1, 0, 1):
                for b in (-1, 0, 1):
                    if (a, b) != (0, 0) and 0 <= k1 + a < m and 0 <= k2 + b < m:
                        assert ((k1 + a) % 2) + 2 * ((k2 + b) % 2) != c


def test_local_order_and_leaf_tiles():
    p = dd.Partition(2, 256, 4, 8, dd.SCHWARZ, leaf_side=8)
    sd = p.subdomains[5]          # interior: 80 x 80 points, 10 x 10 tiles
    assert len(sd.index) == 6400 and len(sd.leaves) == 100
    assert [len(l) for l in sd.levels] == [100, 25, 9, 4, 1]
    lo, hi, st, cnt = sd.leaves[0]
    assert (lo, hi, st, cnt) == ([56, 56], [64, 64], 0, 64)
    # leaves are contiguous in local numbering
    assert all(sd.leaves[i][2] + sd.leaves[i][3] == sd.leaves[i + 1][2] for i in range(99))
    # boundary subdomain: 72 x 72 points, 9 x 9 tiles
    assert len(p.subdomains[0].leaves) == 81


def test_cbd_tree_levels_and_children():
    p = dd.Partition(2, 64, 16, 1, dd.CBD)
    sd = p.subdomains[0]
    assert [len(l) for l in sd.levels] == [64, 16, 4, 1]
    assert sd.root_level == 3
    # level-1 box 0 merges same-color regions (0,0),(1,0),(0,1),(1,1) of the color sub-grid
    assert sd.levels[1][0].children == [0, 1, 8, 9]
    assert sd.levels[1][0].lo == [0, 0] and sd.levels[1][0].hi == [13, 13]
    # every box of a level is the child of exactly one parent
    for l in range(1, len(sd.levels)):
        ch = sorted(c for b in sd.levels[l] for c in b.children)
        assert ch == list(range(len(sd.levels[l - 1])))


def test_single_box_subdomain_is_root():
    p = dd.Partition(2, 16, 2, 1, dd.CBD)
    for sd in p.subdomains:
        assert sd.root_level == 0 and len(sd.levels[0]) == 1


def test_invalid_inputs():
    with pytest.raises(ValueError):
        dd.Partition(2, 30, 4, 1, dd.CBD)
    with pytest.raises(ValueError):
        dd.Partition(2, 32, 8, 3, dd.CBD)

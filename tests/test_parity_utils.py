"""CPU checks of the parity helpers: the tie-band region and the leaf-list
comparison that exempts it."""
import numpy as np
import pytest

import oracle as O
from parity_utils import (band_region, check_block_first, compare_leaf_lists,
                          leaf_of_finest, part1by1, compact1by1)


def test_part1by1_inverts_compact1by1():
    x = np.arange(0, 1 << 12, 7, dtype=np.uint64)
    assert np.array_equal(compact1by1(part1by1(x)), x)
    assert int(part1by1(np.uint64(3))) | (int(part1by1(np.uint64(1))) << 1) == O.morton(3, 1)


def test_band_region_is_cell_and_face_neighbours():
    L = 3
    # level-1 cell (i, j) = (0, 0): itself and its east and north neighbours
    tie = O.zindex(1, 0, 0)
    r = band_region(L, [tie])
    want = np.zeros(1 << (2 * L), dtype=bool)
    for (i, j) in ((0, 0), (1, 0), (0, 1)):
        k = O.zindex(1, i, j) - 1
        want[k * 16:(k + 1) * 16] = True
    assert np.array_equal(r, want)
    assert not band_region(L, []).any()


def test_compare_leaf_lists_exempts_only_the_band():
    L = 2
    uniform = np.arange(5, 21)                          # all finest leaves
    one_coarse = np.array([1] + list(range(9, 21)))     # first quadrant coarse
    compare_leaf_lists(L, uniform, uniform, [], log=lambda *a: None)
    with pytest.raises(AssertionError):
        compare_leaf_lists(L, uniform, one_coarse, [], log=lambda *a: None)
    # a tie on the first level-1 cell explains the difference
    compare_leaf_lists(L, uniform, one_coarse, [1], log=lambda *a: None)
    # a tie far away does not
    with pytest.raises(AssertionError):
        compare_leaf_lists(L, uniform, one_coarse, [4], log=lambda *a: None)
    assert leaf_of_finest(L, one_coarse)[:4].tolist() == [1, 1, 1, 1]


def test_check_block_first_layout():
    """L = 4: quadrant 0 of level 1 is one leaf, the other three quadrants
    are finest (three whole 64-cell blocks).  The block-first list holds the
    blocks, then the coarse leaf; the depth-first list is not block-first,
    and neither is a list with two blocks swapped."""
    L = 4
    off = (4 ** L - 1) // 3
    canon = np.concatenate([[1], off + np.arange(64, 256)])
    stored = np.concatenate([off + np.arange(64, 256), [1]])
    assert check_block_first(L, stored, canon) == 3
    with pytest.raises(AssertionError):
        check_block_first(L, canon, canon)
    swapped = np.concatenate([off + np.arange(128, 192), off + np.arange(64, 128),
                              off + np.arange(192, 256), [1]])
    with pytest.raises(AssertionError):
        check_block_first(L, swapped, canon)
    # a block with one coarse quadrant is not whole: everything stays in order
    canon2 = np.concatenate([off + np.arange(0, 48), [(4 ** 3 - 1) // 3 + 12],
                             off + np.arange(64, 256)])
    stored2 = np.concatenate([off + np.arange(64, 256), off + np.arange(0, 48),
                              [(4 ** 3 - 1) // 3 + 12]])
    assert check_block_first(L, stored2, canon2) == 3

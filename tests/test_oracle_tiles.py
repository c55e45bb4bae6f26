"""Pins of the oracle's block-level redundant layout on grid trees (Sec. 3.5:
data duplicated per thread block instead of per thread, for dense regular
distributions): tiles of grain^3 boxes, one segment per tile holding the rows
of the union of its boxes' near lists.  Checked against the box-grain layout
(grain 1), against box coordinates (tile membership and halos by brute force,
not through the near lists), against hand-counted halo sizes, and by the rows
each near-list entry points at."""
import itertools

import numpy as np
import pytest

import oracle


def _boxes(tree):
    """(instance, box i, j, k) of every leaf, from the anchors (point indices)."""
    return np.concatenate([tree.inst[:, None], tree.anchor // 4], axis=1)


def test_grain_one_is_the_box_grain_layout():
    t = oracle.build_tree_grids([12, 8])
    s, i = oracle.neighbors(t)
    tf, hs, hi, ss, rr = oracle.tile_layout(t, s, i, 1)
    rs, _, S = oracle.red_offsets(t, s, i)
    L = t.n_leaves
    np.testing.assert_array_equal(tf, np.arange(L + 1))
    np.testing.assert_array_equal(hs, s)
    np.testing.assert_array_equal(hi, i)
    np.testing.assert_array_equal(ss, rs)
    # entry e of A: the start of A's segment plus the rows of the entries before it
    occ = np.diff(t.leaf_start)
    for A in range(L):
        rows = rs[A] + np.concatenate([[0], np.cumsum(occ[i[s[A]:s[A + 1]]])[:-1]])
        np.testing.assert_array_equal(rr[s[A]:s[A + 1]], rows)


@pytest.mark.parametrize("grain", [2, 4])
def test_tiles_and_halos_from_box_coordinates(grain):
    sides = [12, 8, 20, 4]        # 3, 2, 5 and 1 boxes per side: partial tiles at the upper faces
    t = oracle.build_tree_grids(sides)
    s, i = oracle.neighbors(t)
    tf, hs, hi, ss, rr = oracle.tile_layout(t, s, i, grain)
    bx = _boxes(t)
    key = [tuple(b[:1]) + tuple(b[1:] // grain) for b in bx]
    # each tile is a run of consecutive boxes sharing one tile key, and no key repeats
    seen = set()
    for tt in range(len(tf) - 1):
        ks = {key[A] for A in range(tf[tt], tf[tt + 1])}
        assert len(ks) == 1 and not (ks & seen)
        seen |= ks
    assert len(seen) == len({*key})
    # halo: every box of the instance within one box of some box of the tile (L-infinity)
    for tt in range(len(tf) - 1):
        mine = bx[tf[tt]:tf[tt + 1]]
        want = [B for B in range(t.n_leaves) if bx[B, 0] == mine[0, 0]
                and np.abs(mine[:, 1:] - bx[B, 1:]).max(axis=1).min() <= 1]
        np.testing.assert_array_equal(hi[hs[tt]:hs[tt + 1]], want)
    # every grid box holds 64 points
    np.testing.assert_array_equal(np.diff(ss), 64 * np.diff(hs))


# Per axis, a tile covering boxes [g i, g i + g - 1] (clipped to the b boxes of the
# side) has a halo of the boxes [g i - 1, g i + g] clipped to [0, b - 1]; summed
# over the tiles of a side by hand:
#   b = 12, g = 2: 3 + 4 + 4 + 4 + 4 + 3 = 22      b = 12, g = 4: 5 + 6 + 5 = 16
#   b = 5,  g = 2: 3 + 4 + 2 = 9                    b = 5,  g = 4: 5 + 2 = 7
#   b = 16, g = 4: 5 + 6 + 6 + 5 = 22               b = 1,  g = 2: 1
# and a cube of b^3 boxes has (per-axis sum)^3 halo boxes over all its tiles.
@pytest.mark.parametrize("n_side,grain,per_axis", [(48, 2, 22), (48, 4, 16), (20, 2, 9), (20, 4, 7),
                                                   (64, 4, 22), (4, 2, 1), (48, 1, 34)])
def test_halo_totals_hand_counted(n_side, grain, per_axis):
    t = oracle.build_tree_grids([n_side])
    s, i = oracle.neighbors(t)
    tf, hs, hi, ss, rr = oracle.tile_layout(t, s, i, grain)
    assert len(hi) == per_axis ** 3
    assert ss[-1] == 64 * per_axis ** 3
    b = n_side // 4
    assert len(tf) - 1 == (-(-b // grain)) ** 3


@pytest.mark.parametrize("grain", [1, 2, 4])
def test_entries_point_at_their_source_rows(grain):
    """The rows at red_row[e] of the tile payload are the sorted rows of the
    entry's source box, for every entry: the layout feeds each target box
    exactly its near sources."""
    sides = [16, 12]
    t = oracle.build_tree_grids(sides)
    s, i = oracle.neighbors(t)
    tf, hs, hi, ss, rr = oracle.tile_layout(t, s, i, grain)
    n = int(sum(v ** 3 for v in sides))
    src = np.arange(n, dtype=np.int64) * 7 + 3          # caller-order rows that name their point
    pay = oracle.restructure_tile_rows(t, hs, hi, ss, src)
    for e in range(len(i)):
        B = i[e]
        np.testing.assert_array_equal(pay[rr[e]:rr[e] + 64], src[t.perm[t.leaf_start[B]:t.leaf_start[B + 1]]])
    # the tile segments hold nothing else: every row is some entry's source row
    assert pay.shape[0] == ss[-1] and len(np.unique(rr)) == len(hi)


@pytest.mark.parametrize("grain", [2, 4])
def test_binding_sizes_the_tile_layout_like_the_oracle(grain):
    """The Python binding sizes the tile-grain buffers from the grids alone
    (per-axis window extents); the oracle's segment total must match it."""
    from paper_2511_21535_amd import api
    from paper_2511_21535_amd import workloads as W
    for sides in ([12, 8, 20, 4], [16], [48, 36, 28], list(W.batched_grid_sides(9, 7))):
        t = oracle.build_tree_grids(sides)
        s, i = oracle.neighbors(t)
        _, _, _, ss, _ = oracle.tile_layout(t, s, i, grain)
        fake = api.Tree(n=0, n_leaves=0, kind=0, key_bits=0, max_level=0, perm=None, leaf_start=None,
                        leaf_key=None, leaf_level=None, iperm=None,
                        grids=[api.Grid(int(n), 1.0 / n, 0.0) for n in sides])
        assert api.tile_entries(fake, grain) == ss[-1], sides

"""Pins of the oracle's keys, trees, near lists, redundant layout and Locality.

Each check compares the oracle against something other than itself: hand
values, closed forms, invariants stated from positions (floating-point cube
geometry), or an index-space characterisation of adjacency.
"""
import numpy as np
import pytest

import oracle
from paper_2511_21535_amd import workloads as W


# ---------------------------------------------------------------- keys ----
def test_morton_hand_values():
    assert oracle.morton3(1, 0, 0, 20) == 1
    assert oracle.morton3(0, 1, 0, 20) == 2
    assert oracle.morton3(0, 0, 1, 20) == 4
    assert oracle.morton3(1, 1, 1, 20) == 7
    assert oracle.morton3(2, 0, 0, 20) == 8
    # x=0b011, y=0b101, z=0b110: digits (x,y,z bits) 0b011, 0b101, 0b110
    assert oracle.morton3(3, 5, 6, 20) == 3 + (5 << 3) + (6 << 6)
    assert oracle.morton3((1 << 20) - 1, (1 << 20) - 1, (1 << 20) - 1, 20) == (1 << 60) - 1


def test_particle_keys_exact_floor_and_domain():
    u = 2.0 ** -20
    x = np.array([u, 0.0, 0.0, 0.5, 1 - 2.0 ** -53, 0.25])
    y = np.array([0.0, u, 0.0, 0.0, 1 - 2.0 ** -53, 0.25])
    z = np.array([0.0, 0.0, u, 0.0, 1 - 2.0 ** -53, 0.25 - 2.0 ** -55])
    key, bad = oracle.particle_keys(x, y, z)
    assert bad == 0
    assert key[0] == 1 and key[1] == 2 and key[2] == 4
    assert key[3] == 1 << 57                      # c_x = 2^19 -> bit 19 of x -> key bit 57
    assert key[4] == (1 << 60) - 1                # floor, never rounds up to 2^20
    # z just below 0.25: c_z = 2^18 - 1
    assert key[5] == oracle.morton3(1 << 18, 1 << 18, (1 << 18) - 1, 20)
    for bad_pt in ([1.0, 0.5, 0.5], [-1e-300, 0.5, 0.5], [np.nan, 0.5, 0.5], [0.5, np.inf, 0.5]):
        _, b = oracle.particle_keys(*[np.array([v]) for v in bad_pt])
        assert b == 1


# ---------------------------------------------------------------- trees ---
def _leaf_of_slot(tree):
    return np.repeat(np.arange(tree.n_leaves), np.diff(tree.leaf_start))


def _cube_bounds(tree):
    lo = tree.anchor.astype(np.float64) * 2.0 ** -20
    hi = (tree.anchor + tree.size[:, None]).astype(np.float64) * 2.0 ** -20
    return lo, hi


@pytest.mark.parametrize("depth", [0, 1, 3])
def test_uniform_tree_closed_form(depth):
    x, y, z, _ = W.uniform_particles(3000, seed=11)
    t = oracle.build_tree_particles(x, y, z, depth=depth, leaf_cap=0)
    # closed form: leaf index per axis = floor(x 2^depth)
    cell = np.stack([np.floor(v * 2 ** depth).astype(np.int64) for v in (x, y, z)], axis=1)
    uniq = np.unique(cell, axis=0)
    assert t.n_leaves == uniq.shape[0]
    assert np.all(t.leaf_level == depth)
    leaf = _leaf_of_slot(t)
    got_cell = t.anchor[leaf] // (1 << (20 - depth))
    np.testing.assert_array_equal(got_cell, cell[t.perm])
    assert np.all(np.diff(t.leaf_key.astype(np.float64)) > 0)


def test_sort_is_stable_on_duplicate_points():
    x = np.array([0.7, 0.1, 0.7, 0.1, 0.7])
    t = oracle.build_tree_particles(x, x, x, depth=2, leaf_cap=0)
    np.testing.assert_array_equal(t.perm, [1, 3, 0, 2, 4])


@pytest.mark.parametrize("cap", [1, 8, 64])
def test_adaptive_tree_invariants(cap):
    x, y, z, _ = W.plummer_mixture(4000, seed=12)
    pos = np.stack([x, y, z], axis=1)
    t = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=cap)
    occ = t.occ
    assert occ.sum() == len(x) and np.all(occ > 0)
    # every leaf holds <= cap points or sits at the depth cap
    assert np.all((occ <= cap) | (t.leaf_level == 20))
    lo, hi = _cube_bounds(t)
    # every particle lies in its leaf's half-open cube (from positions)
    leaf = _leaf_of_slot(t)
    p = pos[t.perm]
    assert np.all((p >= lo[leaf]) & (p < hi[leaf]))
    # the parent of every leaf held more than cap points, counted from positions
    for A in range(t.n_leaves):
        if t.leaf_level[A] == 0:
            continue
        psz = 2 * t.size[A]
        pa = (t.anchor[A] // psz) * psz
        plo, phi = pa * 2.0 ** -20, (pa + psz) * 2.0 ** -20
        inside = np.all((pos >= plo) & (pos < phi), axis=1).sum()
        assert inside > cap
    # leaves are disjoint: sizes are powers of two and anchors are aligned,
    # so disjointness == no anchor inside another leaf's cube
    order = np.argsort(t.leaf_key)
    np.testing.assert_array_equal(order, np.arange(t.n_leaves))


# ---------------------------------------------------------------- near lists
def test_uniform_near_lists_closed_form():
    depth, m = 2, 4
    x, y, z, _ = W.uniform_particles(4096, seed=13)
    t = oracle.build_tree_particles(x, y, z, depth=depth, leaf_cap=0)
    assert t.n_leaves == m ** 3                   # fully occupied
    start, idx = oracle.neighbors(t)
    c = t.anchor // t.size[:, None]
    expect = np.prod(3 - (c == 0) - (c == m - 1), axis=1)
    np.testing.assert_array_equal(np.diff(start), expect)
    assert start[-1] == (3 * m - 2) ** 3
    # index-space characterisation: Chebyshev distance <= 1
    for A in range(t.n_leaves):
        want = np.nonzero(np.max(np.abs(c - c[A]), axis=1) <= 1)[0]
        np.testing.assert_array_equal(idx[start[A]:start[A + 1]], want)


def test_adaptive_near_lists_geometry_and_symmetry():
    x, y, z, _ = W.plummer_mixture(3000, seed=14)
    t = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=16)
    start, idx = oracle.neighbors(t)
    lo, hi = _cube_bounds(t)
    L = t.n_leaves
    near = np.zeros((L, L), dtype=bool)
    for A in range(L):
        near[A, idx[start[A]:start[A + 1]]] = True
        seg = idx[start[A]:start[A + 1]]
        assert np.all(np.diff(seg) > 0) and A in seg
    # L-infinity gap between closed cubes is zero  <=>  near
    gap = np.maximum(0.0, np.maximum(lo[None, :, :] - hi[:, None, :], lo[:, None, :] - hi[None, :, :]))
    np.testing.assert_array_equal(near, np.all(gap == 0.0, axis=2))
    np.testing.assert_array_equal(near, near.T)


def test_grid_tree_and_near_lists():
    sides = np.array([8, 12, 4], dtype=np.int32)
    t = oracle.build_tree_grids(sides)
    nb = sides // 4
    assert t.n_leaves == int((nb ** 3).sum())
    assert np.all(t.occ == 64)
    start, idx = oracle.neighbors(t)
    per_inst = [(3 * m - 2) ** 3 for m in nb]
    tot = np.diff(start)
    for g in range(len(sides)):
        assert tot[t.inst == g].sum() == per_inst[g]
    assert np.all(t.inst[idx] == np.repeat(t.inst, np.diff(start)))
    # points of a box are its 64 grid points, box-major, Morton inside
    off = oracle.grid_offsets(sides)
    for A in (0, 5, t.n_leaves - 1):
        g = t.inst[A]
        pts = t.perm[t.leaf_start[A]:t.leaf_start[A + 1]] - off[g]
        n = sides[g]
        ijk = np.stack([pts % n, (pts // n) % n, pts // (n * n)], axis=1)
        assert np.all(ijk // 4 == t.anchor[A] // 4)
        assert len(set(map(tuple, ijk))) == 64


def test_grid_pair_counts_closed_form():
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
    for n in (16, 48):
        t = oracle.build_tree_grids([n])
        start, idx = oracle.neighbors(t)
        assert oracle.pair_count(t, start, idx) == gold["grid_pair_counts"][str(n)]


# ---------------------------------------------------------------- redundant layout
def test_redundant_payload_from_positions():
    x, y, z, m = W.plummer_mixture(2000, seed=15)
    pos = np.stack([x, y, z], axis=1)
    t = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=32)
    start, idx = oracle.neighbors(t)
    rs, rself, S = oracle.red_offsets(t, start, idx)
    occ = t.occ
    assert S == sum(occ[idx[start[A]:start[A + 1]]].sum() for A in range(t.n_leaves))
    ids = oracle.restructure_rows(t, start, idx, rs, np.arange(len(x), dtype=np.int64))
    lo, hi = _cube_bounds(t)
    for A in range(0, t.n_leaves, 7):
        seg = ids[rs[A]:rs[A + 1]]
        # the sources of A = every particle inside a closed cube that touches A's cube,
        # found from positions: the particle's own leaf cube touches A's
        leaf = np.zeros(len(x), dtype=np.int64)
        leaf[t.perm] = _leaf_of_slot(t)
        gap = np.maximum(0.0, np.maximum(lo[leaf] - hi[A], lo[A] - hi[leaf]))
        want = np.nonzero(np.all(gap == 0.0, axis=1))[0]
        np.testing.assert_array_equal(np.sort(seg), want)
        own = t.perm[t.leaf_start[A]:t.leaf_start[A + 1]]
        np.testing.assert_array_equal(seg[rself[A]:rself[A] + occ[A]], own)
    # payload rows are bit copies
    px = oracle.restructure_rows(t, start, idx, rs, x)
    np.testing.assert_array_equal(px.view(np.uint64), x[ids].view(np.uint64))
    m32 = oracle.restructure_rows(t, start, idx, rs, m.astype(np.float32))
    np.testing.assert_array_equal(m32, m.astype(np.float32)[ids])


# ---------------------------------------------------------------- Locality
def test_locality_hand_values():
    # uniform depth-2 tree, fully occupied: leaf 0 (corner) sees Morton ids 0..7,
    # one run; leaf 1 at (1,0,0) sees {0..8, 10, 12, 14}: four runs
    x, y, z, _ = W.uniform_particles(4096, seed=13)
    t = oracle.build_tree_particles(x, y, z, depth=2, leaf_cap=0)
    start, idx = oracle.neighbors(t)
    np.testing.assert_array_equal(idx[start[1]:start[2]], [0, 1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14])
    for A, runs in ((0, 1), (1, 4)):
        one = oracle.locality(np.array([0, start[A + 1] - start[A]]), idx[start[A]:start[A + 1]],
                              1, 1, 1.0, 1e30)
        assert one["D_mean"] == runs
    # depth-1 tree: every leaf's near list is all 8 leaves -> D = 1, V' = N/S = 1/8
    t1 = oracle.build_tree_particles(x, y, z, depth=1, leaf_cap=0)
    s1, i1 = oracle.neighbors(t1)
    _, _, S = oracle.red_offsets(t1, s1, i1)
    assert S == 8 * len(x)
    loc = oracle.locality(s1, i1, len(x), S, 32.0, cache_bytes=1e12)
    assert loc["D_mean"] == 1.0 and loc["V_ratio"] == 0.125 and loc["locality"] == 0.125


def test_locality_formula_branches():
    """Formula (10) D'V' while the redundant layout fits the cache (V_red <= C,
    the equality included), Formula (11) V'/D' beyond it, on a case where the
    two differ (D' != 1).  One particle at the centre of every leaf of a full
    uniform depth-2 tree (4x4x4 leaves): N = 64, S = (3*4 - 2)^3 = 1000, so
    V' = 64/1000.  The runs of consecutive Morton ids in the 64 near lists,
    counted by hand from the lattice (corner leaves 1 run ... 13 runs for the
    most scattered interior leaves), total 344, so D' = 344/64 = 5.375."""
    c = (np.arange(4) + 0.5) / 4
    x, y, z = (a.ravel() for a in np.meshgrid(c, c, c, indexing="ij"))
    t = oracle.build_tree_particles(x, y, z, depth=2, leaf_cap=0)
    start, idx = oracle.neighbors(t)
    _, _, S = oracle.red_offsets(t, start, idx)
    assert t.n_leaves == 64 and S == 1000
    b = 32.0
    v_red = S * b
    d_p, v_p = 344 / 64, 64 / 1000
    for cache, want in ((1e12, d_p * v_p), (v_red, d_p * v_p),                   # (10): fits, and the edge
                        (v_red - 1.0, v_p / d_p), (1.0, v_p / d_p)):             # (11): exceeds
        loc = oracle.locality(start, idx, 64, S, b, cache_bytes=cache)
        assert loc["D_mean"] == 5.375 and loc["D_ratio"] == 5.375
        assert abs(loc["V_ratio"] - 0.064) <= 1e-15
        assert abs(loc["locality"] - want) <= 1e-15 * want, (cache, loc["locality"], want)
    # the two branches really differ here: 0.344 against about 0.0119
    assert abs(d_p * v_p - 0.344) < 1e-15 and abs(v_p / d_p - 0.011906976744186046) < 1e-15


def test_relative_payload_from_rows_and_centres():
    # the FP32-mixed payload is the bit-copied row minus the target leaf's centre,
    # rounded to single; the centre is the midpoint of the leaf's cube
    x, y, z, m = W.plummer_mixture(3000, 16)
    t = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=32)
    start, idx = oracle.neighbors(t)
    rs, _, S = oracle.red_offsets(t, start, idx)
    p4 = oracle.restructure_gravity_rel(t, start, idx, rs, x, y, z, m)
    lo, hi = _cube_bounds(t)
    centre = 0.5 * (lo + hi)
    owner = np.repeat(np.arange(t.n_leaves), np.diff(rs))
    for d, v in enumerate((x, y, z)):
        rows = oracle.restructure_rows(t, start, idx, rs, v)
        np.testing.assert_array_equal(p4[:, d], (rows - centre[owner, d]).astype(np.float32))
        # relative coordinates stay within the near field of the owner leaf
        span = np.max(t.size) * 2.0 ** -20
        assert np.all(np.abs(p4[:, d]) <= 1.5 * span + 1e-12)
    np.testing.assert_array_equal(p4[:, 3], oracle.restructure_rows(t, start, idx, rs, m).astype(np.float32))


def test_interaction_records_from_segments():
    # the per-interaction records (Sec. 5.2.1) hold, for every near-list entry
    # (A, B), a header (occ_A, occ_B, A, B), A's rows and B's rows; the source
    # part equals B's slice of A's box-grain segment and the target part A's own
    # slice (at red_self), and with the symmetric near relation the records hold
    # E headers plus 2 S rows
    x, y, z, m = W.plummer_mixture(2500, 17)
    t = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=24)
    start, idx = oracle.neighbors(t)
    rs, rself, S = oracle.red_offsets(t, start, idx)
    E = len(idx)
    occ = np.diff(t.leaf_start)
    rec8, r8 = oracle.restructure_interactions(t, start, idx, x, y, z, m, prec="fp64")
    rec4, r4 = oracle.restructure_interactions(t, start, idx, x, y, z, m, prec="fp32")
    np.testing.assert_array_equal(rec8, rec4)
    assert rec8[-1] == E + 2 * S == len(r8) == len(r4)
    seg8 = oracle.restructure_rows(t, start, idx, rs, np.stack([x, y, z, m], 1))
    seg4 = oracle.restructure_gravity_rel(t, start, idx, rs, x, y, z, m)
    lo, hi = _cube_bounds(t)
    for A in range(t.n_leaves):
        off = rs[A]
        for e in range(start[A], start[A + 1]):
            B = idx[e]
            r = rec8[e]
            assert list(r8[r]) == [occ[A], occ[B], A, B]
            assert list(r4[r].view(np.int32)) == [occ[A], occ[B], A, B]
            tgt8, src8 = r8[r + 1:r + 1 + occ[A]], r8[r + 1 + occ[A]:r + 1 + occ[A] + occ[B]]
            np.testing.assert_array_equal(src8, seg8[off:off + occ[B]])
            np.testing.assert_array_equal(tgt8, seg8[rs[A] + rself[A]:rs[A] + rself[A] + occ[A]])
            np.testing.assert_array_equal(r4[r + 1 + occ[A]:r + 1 + occ[A] + occ[B]], seg4[off:off + occ[B]])
            np.testing.assert_array_equal(r4[r + 1:r + 1 + occ[A]],
                                          seg4[rs[A] + rself[A]:rs[A] + rself[A] + occ[A]])
            # the targets lie in A's cube (geometry, independent of the segments)
            assert np.all((tgt8[:, :3] >= lo[A]) & (tgt8[:, :3] < hi[A]))
            off += occ[B]

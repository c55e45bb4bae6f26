"""Pins of the oracle's periodic near field (the periodic interactions of the
stellar-dynamics case, Sec. 5.2, on the unit torus).

What fixes each value, other than the oracle itself: the symmetry of the
torus adjacency (B seen from A through image c iff A seen from B through the
opposite image), agreement with the plain lists away from the boundary, a
lattice whose every particle sees the same neighbourhood (equal potentials,
zero forces), invariance under a translation by half the domain (which maps
the octree onto itself), momentum conservation, central finite differences
for the adjoint, and sums recomputed from the laid-out rows.
"""
import numpy as np
import pytest

import oracle
from paper_2511_21535_amd import workloads as W


def _lists(nb):
    start, idx, sh = nb
    return [set(zip(idx[start[a]:start[a + 1]].tolist(), sh[start[a]:start[a + 1]].tolist()))
            for a in range(start.shape[0] - 1)]


def _dyadic(v, bits=30):
    return np.floor(v * 2.0 ** bits) / 2.0 ** bits


@pytest.fixture(scope="module")
def clustered():
    x, y, z, m = W.plummer_mixture(600, seed=71)
    x, y, z = (_dyadic(v) for v in (x, y, z))
    t = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=8)
    return x, y, z, m, t, oracle.neighbors_periodic(t)


def test_periodic_lists_symmetric_sorted_and_interior(clustered):
    x, y, z, m, t, nb = clustered
    start, idx, sh = nb
    L = t.n_leaves
    sets = _lists(nb)
    for a in range(L):
        e = slice(start[a], start[a + 1])
        keys = sh[e].astype(np.int64) * L + idx[e]
        assert np.all(np.diff(keys) > 0)                   # ascending (code, B), no repeats
        assert (a, 13) in sets[a]
        for b, c in sets[a]:
            assert (a, 26 - c) in sets[b]
    # a leaf whose neighbourhood stays inside the domain has the plain list
    ps, pi = oracle.neighbors(t)
    dim = 1 << 20
    inner = 0
    for a in range(L):
        lo, s = t.anchor[a], t.size[a]
        if np.all(lo - s >= 0) and np.all(lo + 2 * s <= dim):
            # its neighbours all lie in the closed 3x3x3 block, which does not wrap
            assert sets[a] == {(int(b), 13) for b in pi[ps[a]:ps[a + 1]]}
            inner += 1
    assert inner > 0


def test_periodic_lattice_equal_potentials_zero_forces():
    # one particle at the centre of every leaf of a uniform depth-3 tree: on the
    # torus every particle sees the same 26 neighbours, placed symmetrically
    k = (np.arange(8) + 0.5) / 8
    gx, gy, gz = np.meshgrid(k, k, k, indexing="ij")
    x, y, z = gx.ravel(), gy.ravel(), gz.ravel()
    m = np.ones_like(x)
    t = oracle.build_tree_particles(x, y, z, depth=3, leaf_cap=0)
    nb = oracle.neighbors_periodic(t)
    assert np.all(np.diff(nb[0]) == 27)
    phi, ax, ay, az = oracle.gravity(x, y, z, m, 1e-3, t, nb)
    # the 26 neighbours at distances h, h sqrt2, h sqrt3 (h = 1/8), softened
    h, e2 = 1 / 8, 1e-6
    want = -(6 / np.sqrt(h * h + e2) + 12 / np.sqrt(2 * h * h + e2) + 8 / np.sqrt(3 * h * h + e2))
    np.testing.assert_allclose(phi, want, rtol=1e-13)
    for a in (ax, ay, az):
        assert np.abs(a).max() <= 1e-12 * 6 / h ** 2
    # without images the boundary particles are pulled inwards
    p2 = oracle.gravity(x, y, z, m, 1e-3, t)
    assert np.abs(p2[1]).max() > 1.0


def test_periodic_translation_by_half_domain(clustered):
    x, y, z, m, t, nb = clustered
    res = oracle.gravity(x, y, z, m, 1e-3, t, nb)
    xs = np.mod(x + 0.5, 1.0)                              # exact: 30-bit dyadic positions
    ts = oracle.build_tree_particles(xs, y, z, depth=20, leaf_cap=8)
    assert ts.n_leaves == t.n_leaves
    res_s = oracle.gravity(xs, y, z, m, 1e-3, ts, oracle.neighbors_periodic(ts))
    for a, b in zip(res, res_s):
        np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-12 * np.abs(a).max())
    # the plain near field is not invariant: the test can see a missing image
    plain_s = oracle.gravity(xs, y, z, m, 1e-3, ts)
    assert np.abs(plain_s[1] - res[1]).max() > 1e-6 * np.abs(res[1]).max()


def test_periodic_momentum_conservation(clustered):
    x, y, z, m, t, nb = clustered
    phi, ax, ay, az = oracle.gravity(x, y, z, m, 1e-3, t, nb)
    for a in (ax, ay, az):
        assert abs(np.dot(m, a)) <= 1e-12 * np.dot(m, np.abs(a))


def test_periodic_adjoint_finite_differences():
    x, y, z, m = W.plummer_mixture(150, seed=72)
    t = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=8)
    nb = oracle.neighbors_periodic(t)
    gp, gax, gay, gaz = (W.normal_like(150, seed=s) for s in (73, 74, 75, 76))
    eps = 1e-3

    def loss(x, y, z, m):
        phi, ax, ay, az = oracle.gravity(x, y, z, m, eps, t, nb)
        return np.sum(gp * phi) + np.sum(gax * ax) + np.sum(gay * ay) + np.sum(gaz * az)

    gm, gx, gy, gz = oracle.gravity_adjoint(x, y, z, m, eps, gp, gax, gay, gaz, t, nb)
    assert abs(np.dot(m, gm) - loss(x, y, z, m)) < 1e-12 * abs(loss(x, y, z, m))
    # pick particles whose leaf has a shifted image in its list
    start, idx, sh = nb
    leaf_of = np.empty(150, dtype=np.int64)
    for a in range(t.n_leaves):
        leaf_of[t.perm[t.leaf_start[a]:t.leaf_start[a + 1]]] = a
    wrapped = [j for j in range(150) if np.any(sh[start[leaf_of[j]]:start[leaf_of[j] + 1]] != 13)]
    assert len(wrapped) >= 8
    h = 1e-6
    scale = max(np.abs(gx).max(), np.abs(gy).max(), np.abs(gz).max())
    for j in wrapped[:8]:
        for idx_ax, grad in ((0, gx), (1, gy), (2, gz)):
            xp = [x.copy(), y.copy(), z.copy()]
            xm = [x.copy(), y.copy(), z.copy()]
            xp[idx_ax][j] += h
            xm[idx_ax][j] -= h
            fd = (loss(*xp, m) - loss(*xm, m)) / (2 * h)
            assert abs(fd - grad[j]) <= 1e-5 * scale


def test_periodic_layouts_reproduce_the_sum(clustered):
    x, y, z, m, t, nb = clustered
    start, idx, sh = nb
    rs, rself, S = oracle.red_offsets(t, start, idx, sh)
    rows = oracle.restructure_gravity_rows(t, start, idx, rs, x, y, z, m, sh)
    rel = oracle.restructure_gravity_rel(t, start, idx, rs, x, y, z, m, sh)
    # the rows of each segment are the listed images, in list order
    shift = oracle.shift_vectors(sh)
    k = 0
    for a in range(t.n_leaves):
        c = (t.anchor[a] + t.size[a] / 2.0) / 2.0 ** 20
        for e in range(start[a], start[a + 1]):
            b = idx[e]
            j = t.perm[t.leaf_start[b]:t.leaf_start[b + 1]]
            want = np.stack([x[j] + shift[e, 0], y[j] + shift[e, 1], z[j] + shift[e, 2], m[j]], 1)
            np.testing.assert_array_equal(rows[k:k + len(j)], want)
            np.testing.assert_array_equal(rel[k:k + len(j), :3],
                                          (want[:, :3] - c).astype(np.float32))
            if b == a and sh[e] == 13:
                assert rself[a] == k - rs[a]
            k += len(j)
    assert k == S
    # direct sums over each segment give the periodic near field
    phi = np.zeros_like(x)
    for a in range(t.n_leaves):
        seg = rows[rs[a]:rs[a + 1]]
        tg = t.perm[t.leaf_start[a]:t.leaf_start[a + 1]]
        for u, i in enumerate(tg):
            d = seg[:, :3] - np.array([x[i], y[i], z[i]])
            w = seg[:, 3] / np.sqrt(np.sum(d * d, 1) + 1e-6)
            w[rself[a] + u] = 0.0
            phi[i] = -np.sum(w)
    np.testing.assert_allclose(phi, oracle.gravity(x, y, z, m, 1e-3, t, nb)[0], rtol=1e-12)
    # per-interaction records carry the source image
    rec, r8 = oracle.restructure_interactions(t, start, idx, x, y, z, m, "fp64", nbr_shift=sh)
    for e in range(0, idx.shape[0], 7):
        a = np.searchsorted(start, e, side="right") - 1
        b = idx[e]
        oa = t.leaf_start[a + 1] - t.leaf_start[a]
        j = t.perm[t.leaf_start[b]:t.leaf_start[b + 1]]
        got = r8[rec[e] + 1 + oa:rec[e] + 1 + oa + len(j)]
        np.testing.assert_array_equal(got[:, 0], x[j] + shift[e, 0])
        np.testing.assert_array_equal(got[:, 2], z[j] + shift[e, 2])

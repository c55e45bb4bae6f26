"""Pins of the oracle's remote near field (the remote interactions of the
stellar-dynamics case, Sec. 5.2: targets of one domain, sources received from
another).

What fixes each value, other than the oracle itself: a source set identical to
the target set (remote lists are then the plain lists, and every potential
gains exactly the point's own copy at distance zero, -m_i / eps, with the
forces unchanged); two sets on uniform trees of one depth, whose leaves are the
occupied cells of one grid, so the near field of a point in their union is its
near field in its own set plus its remote near field in the other (also on the
torus); and the symmetry of the cross relation.
"""
import numpy as np
import pytest

import oracle
from paper_2511_21535_amd import workloads as W


def _sets():
    a = W.uniform_particles(700, seed=81)
    b = W.plummer_mixture(900, seed=82)
    return a, b


def test_remote_identical_copy():
    x, y, z, m = W.plummer_mixture(800, seed=83)
    t = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=8)
    eps = 1e-3
    for periodic in (False, True):
        nb = oracle.neighbors_remote(t, t, periodic)
        plain = oracle.neighbors_periodic(t) if periodic else oracle.neighbors(t)
        for u, v in zip(nb, plain):
            np.testing.assert_array_equal(u, v)
        loc = oracle.gravity(x, y, z, m, eps, t, oracle.neighbors_periodic(t) if periodic else None)
        rem = oracle.gravity_remote(x, y, z, t, x, y, z, m, t, eps, nb)
        np.testing.assert_allclose(rem[0], loc[0] - m / eps, rtol=1e-12)
        for a, b in zip(rem[1:], loc[1:]):
            np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("periodic", [False, True])
def test_remote_completes_the_union_on_uniform_trees(periodic):
    (xa, ya, za, ma), (xb, yb, zb, mb) = _sets()
    depth, eps = 3, 1e-3
    ta = oracle.build_tree_particles(xa, ya, za, depth=depth, leaf_cap=0)
    tb = oracle.build_tree_particles(xb, yb, zb, depth=depth, leaf_cap=0)
    xu, yu, zu, mu = (np.concatenate(p) for p in ((xa, xb), (ya, yb), (za, zb), (ma, mb)))
    tu = oracle.build_tree_particles(xu, yu, zu, depth=depth, leaf_cap=0)
    union = oracle.gravity(xu, yu, zu, mu, eps, tu, oracle.neighbors_periodic(tu) if periodic else None)
    loc = oracle.gravity(xa, ya, za, ma, eps, ta, oracle.neighbors_periodic(ta) if periodic else None)
    rem = oracle.gravity_remote(xa, ya, za, ta, xb, yb, zb, mb, tb, eps,
                                oracle.neighbors_remote(ta, tb, periodic))
    n = len(xa)
    for u, l_, r_ in zip(union, loc, rem):
        np.testing.assert_allclose(l_ + r_, u[:n], rtol=1e-12, atol=1e-12 * np.abs(u[:n]).max())
    # the remote part is not negligible: the test can see a missing source
    assert np.abs(rem[0]).max() > 0.1 * np.abs(loc[0]).max()


def test_remote_lists_symmetric():
    (xa, ya, za, _), (xb, yb, zb, _) = _sets()
    ta = oracle.build_tree_particles(xa, ya, za, depth=20, leaf_cap=8)
    tb = oracle.build_tree_particles(xb, yb, zb, depth=20, leaf_cap=8)
    for periodic in (False, True):
        sa, ia, ca = oracle.neighbors_remote(ta, tb, periodic)
        sb, ib, cb = oracle.neighbors_remote(tb, ta, periodic)
        ab = {(A, int(ia[e]), int(ca[e])) for A in range(ta.n_leaves) for e in range(sa[A], sa[A + 1])}
        ba = {(int(ib[e]), B, 26 - int(cb[e])) for B in range(tb.n_leaves) for e in range(sb[B], sb[B + 1])}
        assert ab == ba and len(ab) > 0
        for A in range(ta.n_leaves):
            keys = ca[sa[A]:sa[A + 1]].astype(np.int64) * tb.n_leaves + ia[sa[A]:sa[A + 1]]
            assert np.all(np.diff(keys) > 0)

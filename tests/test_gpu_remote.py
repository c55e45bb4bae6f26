"""GPU parity of remote interactions (targets of one particle set, sources of
another with its own tree, Sec. 5.2) against the FP64 oracle, through the C ABI.

Bit-exact: the remote lists with their image codes, S, the segment offsets and
the payload.  Floating point: relative L2 <= 1e-12 (FP64), <= 1e-5 (FP32-mixed).
The remote sums are added to the outputs: after the local evaluation they
complete the near field, checked against the union of the two sets on uniform
trees.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_21535_amd import api
from paper_2511_21535_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
DEV = "cuda"


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def _n(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _split(n, seed):
    """One Plummer mixture cut at x = 0.5: the targets' domain and the other one."""
    x, y, z, m = W.plummer_mixture(n, seed)
    a = x < 0.5
    return tuple(v[a].copy() for v in (x, y, z, m)), tuple(v[~a].copy() for v in (x, y, z, m))


CASES = [(6000, 91, 16), (3000, 92, 1), (20000, 93, 64)]


@pytest.mark.parametrize("n,seed,cap", CASES)
@pytest.mark.parametrize("periodic", [False, True])
def test_remote_lists_layout_and_sums(n, seed, cap, periodic):
    (xa, ya, za, ma), (xb, yb, zb, mb) = _split(n, seed)
    print(f"case remote n={n} seed={seed} cap={cap} periodic={periodic}", flush=True)
    ga, gb = [_t(v) for v in (xa, ya, za, ma)], [_t(v) for v in (xb, yb, zb, mb)]
    ta = api.Tree.build_particles(*ga[:3], depth=20, leaf_cap=cap)
    tb = api.Tree.build_particles(*gb[:3], depth=20, leaf_cap=cap)
    nb = api.build_neighbors(ta, periodic=periodic, src_tree=tb)
    ota = oracle.build_tree_particles(xa, ya, za, depth=20, leaf_cap=cap)
    otb = oracle.build_tree_particles(xb, yb, zb, depth=20, leaf_cap=cap)
    ref_nb = oracle.neighbors_remote(ota, otb, periodic)
    np.testing.assert_array_equal(_n(nb.nbr_start), ref_nb[0])
    np.testing.assert_array_equal(_n(nb.nbr_idx), ref_nb[1])
    if periodic:
        np.testing.assert_array_equal(_n(nb.nbr_shift), ref_nb[2])
    assert nb.count > 0
    ref = oracle.gravity_remote(xa, ya, za, ota, xb, yb, zb, mb, otb, 1e-3, ref_nb)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32)):
        rs, rows = oracle.restructure_remote(ota, otb, ref_nb, xb, yb, zb, mb, prec=prec)
        assert nb.red_entries == len(rows)
        red = api.restructure_remote(ta, tb, nb, *gb, prec=prec)
        assert red.count == len(rows)
        np.testing.assert_array_equal(_n(red.red_start), rs)
        assert np.all(_n(red.red_self)[:ta.n_leaves] == -1)
        view = np.uint64 if prec == "fp64" else np.uint32
        np.testing.assert_array_equal(_n(red.planes[0])[:len(rows)].view(view), rows.view(view))
        for layout in ("gather", "redundant"):
            o = [_n(v) for v in api.gravity_remote(ta, tb, nb, 1e-3, *ga[:3], *gb, layout=layout, prec=prec,
                                                   red=red)]
            e_phi, e_a = _rel(o[0], ref[0]), _rel(np.stack(o[1:]), np.stack(ref[1:]))
            print(f"  {prec} {layout}: phi {e_phi:.2e} a {e_a:.2e}", flush=True)
            assert e_phi <= tol and e_a <= tol


@pytest.mark.parametrize("periodic", [False, True])
def test_local_plus_remote_is_the_union(periodic):
    """Uniform trees of one depth: the local sums of one set plus its remote
    sums over the other (added to the same outputs on the GPU) equal the near
    field of the union."""
    xa, ya, za, ma = W.uniform_particles(3000, seed=94)
    xb, yb, zb, mb = W.plummer_mixture(4000, seed=95)
    depth = 4
    ga, gb = [_t(v) for v in (xa, ya, za, ma)], [_t(v) for v in (xb, yb, zb, mb)]
    ta = api.Tree.build_particles(*ga[:3], depth=depth, leaf_cap=0)
    tb = api.Tree.build_particles(*gb[:3], depth=depth, leaf_cap=0)
    xu, yu, zu, mu = (np.concatenate(p) for p in ((xa, xb), (ya, yb), (za, zb), (ma, mb)))
    tu = oracle.build_tree_particles(xu, yu, zu, depth=depth, leaf_cap=0)
    union = oracle.gravity(xu, yu, zu, mu, 1e-3, tu, oracle.neighbors_periodic(tu) if periodic else None)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32)):
        out = api.gravity(ta, ta.neighbors(periodic=periodic), 1e-3, *ga, prec=prec)
        nb = api.build_neighbors(ta, periodic=periodic, src_tree=tb)
        red = api.restructure_remote(ta, tb, nb, *gb, prec=prec)
        api.gravity_remote(ta, tb, nb, 1e-3, *ga[:3], layout="redundant", prec=prec, red=red, out=list(out))
        o = [_n(v) for v in out]
        ref = [u[:len(xa)] for u in union]
        assert _rel(o[0], ref[0]) <= tol and _rel(np.stack(o[1:]), np.stack(ref[1:])) <= tol


def _fill(n, v):
    return [torch.full((n,), v, dtype=torch.float64, device=DEV) for _ in range(4)]


def test_remote_edge_cases():
    """Sets whose trees do not touch (plain: no remote entry, outputs kept;
    periodic: they meet across the domain's face x = 0), an empty source set, an
    empty target set, and one point against one point (the closed form)."""
    rng = np.random.default_rng(96)
    # slabs x < 0.2 and x >= 0.75: their leaves (at most 8 points each) stay
    # inside x <= 0.25 and x >= 0.75, so only the images across x = 0 meet
    A = rng.random((500, 3))
    A[:, 0] *= 0.2
    B = rng.random((700, 3))
    B[:, 0] = 0.75 + 0.25 * B[:, 0]
    mb = rng.uniform(0.5, 1.5, 700)
    ga = [_t(A[:, d].copy()) for d in range(3)]
    gb = [_t(B[:, d].copy()) for d in range(3)] + [_t(mb)]
    ta = api.Tree.build_particles(*ga, depth=20, leaf_cap=8)
    tb = api.Tree.build_particles(*gb[:3], depth=20, leaf_cap=8)
    ota = oracle.build_tree_particles(A[:, 0], A[:, 1], A[:, 2], depth=20, leaf_cap=8)
    otb = oracle.build_tree_particles(B[:, 0], B[:, 1], B[:, 2], depth=20, leaf_cap=8)
    print("case remote apart", flush=True)
    nb = api.build_neighbors(ta, src_tree=tb)
    assert nb.count == 0 and nb.red_entries == 0
    assert np.all(_n(nb.nbr_start) == 0)
    for prec in ("fp64", "fp32"):
        red = api.restructure_remote(ta, tb, nb, *gb, prec=prec)
        assert red.count == 0
        for layout in ("gather", "redundant"):
            out = api.gravity_remote(ta, tb, nb, 1e-3, *ga, *gb, layout=layout, prec=prec, red=red,
                                     out=_fill(500, 1.5))
            assert all(np.all(_n(o) == 1.5) for o in out)
    print("case remote apart periodic", flush=True)
    nb = api.build_neighbors(ta, periodic=True, src_tree=tb)
    ref_nb = oracle.neighbors_remote(ota, otb, True)
    assert nb.count == len(ref_nb[1]) > 0
    np.testing.assert_array_equal(_n(nb.nbr_idx), ref_nb[1])
    np.testing.assert_array_equal(_n(nb.nbr_shift), ref_nb[2])
    assert np.all(ref_nb[2] != 13)
    ref = oracle.gravity_remote(A[:, 0], A[:, 1], A[:, 2], ota, B[:, 0], B[:, 1], B[:, 2], mb, otb, 1e-3, ref_nb)
    red = api.restructure_remote(ta, tb, nb, *gb, prec="fp64")
    for layout in ("gather", "redundant"):
        o = [_n(v) for v in api.gravity_remote(ta, tb, nb, 1e-3, *ga, *gb, layout=layout, red=red)]
        assert _rel(o[0], ref[0]) <= TOL64 and _rel(np.stack(o[1:]), np.stack(ref[1:])) <= TOL64

    print("case remote empty sources", flush=True)
    e = _t(np.zeros(0))
    te = api.Tree.build_particles(e, e, e)
    nb = api.build_neighbors(ta, src_tree=te)
    assert nb.count == 0 and nb.red_entries == 0
    red = api.restructure_remote(ta, te, nb, e, e, e, e, prec="fp32")
    for layout in ("gather", "redundant"):
        out = api.gravity_remote(ta, te, nb, 1e-3, *ga, e, e, e, e, layout=layout, prec="fp32", red=red,
                                 out=_fill(500, -2.0))
        assert all(np.all(_n(o) == -2.0) for o in out)

    print("case remote empty targets", flush=True)
    nb = api.build_neighbors(te, src_tree=tb)
    assert nb.count == 0 and _n(nb.nbr_start).tolist() == [0]
    red = api.restructure_remote(te, tb, nb, *gb, prec="fp64")
    assert red.count == 0
    out = api.gravity_remote(te, tb, nb, 1e-3, e, e, e, *gb, layout="gather")
    assert all(o.numel() == 0 for o in out)

    print("case remote one point each", flush=True)
    p, q, mq, eps = np.array([0.3, 0.4, 0.5]), np.array([0.35, 0.38, 0.51]), 0.75, 1e-3
    gp = [_t(np.array([v])) for v in p]
    gq = [_t(np.array([v])) for v in q] + [_t(np.array([mq]))]
    tp = api.Tree.build_particles(*gp, depth=20, leaf_cap=64)
    tq = api.Tree.build_particles(*gq[:3], depth=20, leaf_cap=64)
    nb = api.build_neighbors(tp, src_tree=tq)
    assert nb.count == 1 and nb.red_entries == 1
    d = p - q
    w = 1.0 / np.sqrt(d @ d + eps * eps)
    want = np.array([-mq * w, *(-mq * w ** 3 * d)])
    for prec, tol in (("fp64", 1e-14), ("fp32", TOL32)):
        red = api.restructure_remote(tp, tq, nb, *gq, prec=prec)
        for layout in ("gather", "redundant"):
            got = np.array([_n(v)[0] for v in api.gravity_remote(tp, tq, nb, eps, *gp, *gq, layout=layout,
                                                                 prec=prec, red=red)])
            np.testing.assert_allclose(got, want, rtol=tol)


@pytest.mark.slow
def test_remote_full_size_plummer_2m_cut():
    """The 2^21-particle Plummer workload cut at x = 0.5 into two domains with
    trees of their own, FP32-mixed, as the benchmark times it: the whole plain
    remote lists bit-exact and every remote sum; on the torus, sampled target
    leaves (at the cut, at the face x = 0 and elsewhere)."""
    w = W.WORKLOADS["gravity_plummer_2m"]
    x, y, z, m = W.particles("gravity_plummer_2m")
    cut = x < 0.5
    a = [v[cut].copy() for v in (x, y, z, m)]
    b = [v[~cut].copy() for v in (x, y, z, m)]
    print("case remote gravity_plummer_2m cut: building", flush=True)
    ga, gb = [_t(v) for v in a], [_t(v) for v in b]
    ta = api.Tree.build_particles(*ga[:3], depth=w["depth"], leaf_cap=w["leaf_cap"])
    tb = api.Tree.build_particles(*gb[:3], depth=w["depth"], leaf_cap=w["leaf_cap"])
    ota = oracle.build_tree_particles(*a[:3], depth=w["depth"], leaf_cap=w["leaf_cap"])
    otb = oracle.build_tree_particles(*b[:3], depth=w["depth"], leaf_cap=w["leaf_cap"])
    np.testing.assert_array_equal(_n(ta.leaf_start), ota.leaf_start)
    np.testing.assert_array_equal(_n(tb.leaf_start), otb.leaf_start)
    nb = api.build_neighbors(ta, src_tree=tb)
    ref_nb = oracle.neighbors_remote(ota, otb, False)
    np.testing.assert_array_equal(_n(nb.nbr_start), ref_nb[0])
    np.testing.assert_array_equal(_n(nb.nbr_idx), ref_nb[1])
    ref = oracle.gravity_remote(*a[:3], ota, *b, otb, w["eps"], ref_nb)
    red = api.restructure_remote(ta, tb, nb, *gb, prec="fp32")
    for layout in ("gather", "redundant"):
        o = [_n(v) for v in api.gravity_remote(ta, tb, nb, w["eps"], *ga[:3], *gb, layout=layout, prec="fp32",
                                               red=red)]
        e_phi, e_a = _rel(o[0], ref[0]), _rel(np.stack(o[1:]), np.stack(ref[1:]))
        print(f"  fp32 {layout}: phi {e_phi:.2e} a {e_a:.2e}", flush=True)
        assert e_phi <= TOL32 and e_a <= TOL32

    print("case remote gravity_plummer_2m cut, periodic: sampled leaves", flush=True)
    nb = api.build_neighbors(ta, periodic=True, src_tree=tb)
    rng = np.random.default_rng(1)
    lo = ota.anchor[:, 0]
    hi = lo + ota.size
    face = np.flatnonzero((lo == 0) | (hi == 1 << 19))
    sel = np.unique(np.concatenate([rng.choice(face, 96, replace=False),
                                    rng.choice(ota.n_leaves, 32, replace=False), [0, ota.n_leaves - 1]]))
    ss, si, ssh = oracle.neighbors_remote(ota, otb, True, sel)
    assert np.any(ssh != 13) and np.any(ssh == 13)
    gs, gi, gsh = _n(nb.nbr_start), _n(nb.nbr_idx), _n(nb.nbr_shift)
    for k, A in enumerate(sel):
        np.testing.assert_array_equal(gi[gs[A]:gs[A + 1]], si[ss[k]:ss[k + 1]])
        np.testing.assert_array_equal(gsh[gs[A]:gs[A + 1]], ssh[ss[k]:ss[k + 1]])
    # the sampled lists as a whole-tree CSR (other leaves empty) for the oracle's sums
    counts = np.zeros(ota.n_leaves, dtype=np.int64)
    counts[sel] = np.diff(ss)
    full = (np.concatenate([[0], np.cumsum(counts)]).astype(np.int64), si, ssh)
    ref = oracle.gravity_remote(*a[:3], ota, *b, otb, w["eps"], full)
    idx = np.concatenate([ota.perm[ota.leaf_start[A]:ota.leaf_start[A + 1]] for A in sel])
    red = api.restructure_remote(ta, tb, nb, *gb, prec="fp32")
    for layout in ("gather", "redundant"):
        o = [_n(v)[idx] for v in api.gravity_remote(ta, tb, nb, w["eps"], *ga[:3], *gb, layout=layout,
                                                    prec="fp32", red=red)]
        r = [v[idx] for v in ref]
        e_phi, e_a = _rel(o[0], r[0]), _rel(np.stack(o[1:]), np.stack(r[1:]))
        print(f"  fp32 {layout}: phi {e_phi:.2e} a {e_a:.2e}", flush=True)
        assert e_phi <= TOL32 and e_a <= TOL32

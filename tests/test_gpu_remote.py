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

"""p2p_eval_gravity_noalloc (the entry point that allocates nothing) against
p2p_eval_gravity through the C ABI: two calls in a row on one GPU, the second
on a smaller input, each bit-identical to the workspace entry point (the same
kernels on the same rows) and, on the small case, within 1e-12 of the FP64
oracle; both layouts and precisions; sizes beyond the static scratch refused
before any work."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2511_21535_amd import _lib as L
from paper_2511_21535_amd import api
from paper_2511_21535_amd import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"
EPS = 1e-3


def _setup(x, y, z, m, depth, leaf_cap):
    t = [torch.as_tensor(v, device=DEV) for v in (x, y, z, m)]
    tree = api.Tree.build_particles(t[0], t[1], t[2], depth=depth, leaf_cap=leaf_cap)
    return t, tree, tree.neighbors()


def _poisoned(n):
    return [torch.full((n,), float("nan"), dtype=torch.float64, device=DEV) for _ in range(4)]


def _both(t, tree, nbrs, layout, prec, red=None):
    ref = api.gravity(tree, nbrs, EPS, *t, layout=layout, prec=prec, red=red)
    got = api.gravity_noalloc(tree, nbrs, EPS, *t, layout=layout, prec=prec, red=red, out=_poisoned(tree.n))
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    return got


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_workspace_entry_twice(prec):
    # first call: 2^18 particles of a Plummer mixture, adaptive tree (leaf cap 64)
    print(f"case noalloc first call n=2^18 prec={prec}", flush=True)
    x, y, z, m = W.plummer_mixture(1 << 18, seed=7)
    t, tree, nbrs = _setup(x, y, z, m, depth=20, leaf_cap=64)
    _both(t, tree, nbrs, "gather", prec)
    red = api.restructure_gravity(tree, nbrs, *t, prec=prec)
    _both(t, tree, nbrs, "redundant", prec, red=red)
    # second call, smaller: 4096 uniform particles, depth-3 tree; the scratch
    # still holds the first call's rows beyond row 4096
    print(f"case noalloc second call n=4096 prec={prec}", flush=True)
    x2, y2, z2, m2 = W.uniform_particles(4096, seed=1)
    t2, tree2, nbrs2 = _setup(x2, y2, z2, m2, depth=3, leaf_cap=0)
    got = _both(t2, tree2, nbrs2, "gather", prec)
    ot = oracle.build_tree_particles(x2, y2, z2, depth=3, leaf_cap=0)
    want = oracle.gravity(x2, y2, z2, m2, EPS, ot)
    tol = 1e-12 if prec == "fp64" else 1e-5
    for a, b in zip(got, want):
        a = a.cpu().numpy()
        assert np.linalg.norm(a - b) / np.linalg.norm(b) <= tol


def test_noalloc_refuses_beyond_scratch():
    # a tree struct that claims 2^21 + 1 points: refused on the host before any
    # launch (the arrays are never read)
    print("case noalloc refuses n=2^21+1", flush=True)
    x, y, z, m = W.uniform_particles(4096, seed=3)
    t, tree, nbrs = _setup(x, y, z, m, depth=3, leaf_cap=0)
    ts, ns = tree.struct(), nbrs.struct()
    ts.n = (1 << 21) + 1
    ts.n_leaves = tree.n_leaves
    out = _poisoned(tree.n)
    st = L.load().p2p_eval_gravity_noalloc(ctypes.byref(ts), ctypes.byref(ns), None, L.P2P_GATHER, L.P2P_FP64,
                                           EPS, *[ctypes.c_void_p(v.data_ptr()) for v in t],
                                           *[ctypes.c_void_p(o.data_ptr()) for o in out],
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == L.P2P_EUNSUPPORTED
    assert b"static scratch" in L.load().p2p_last_error()
    torch.cuda.synchronize()
    assert all(torch.isnan(o).all() for o in out)

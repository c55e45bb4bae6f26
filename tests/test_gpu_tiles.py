"""Tile-grain redundant layout on grid trees (per-block redundancy, Sec. 3.5)
against the oracle: the layout bit for bit (segment starts, the row of every
near-list entry, the payload) and the evaluation from it on every Helmholtz
path (single RHS and multi-RHS on the matrix cores, ragged RHS counts, FP64),
including partial tiles at the upper faces and instances of one box."""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_21535_amd import api
from paper_2511_21535_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
DEV = "cuda"


def _n(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _tree(sides):
    grids = [api.Grid(int(s), *W.grid_geometry(int(s))) for s in sides]
    gt = api.Tree.build_grids(grids, device=DEV)
    return gt, gt.neighbors()


def _check_layout(gt, gn, red, sides, grain, q):
    ot = oracle.build_tree_grids(sides)
    os_, oi = oracle.neighbors(ot)
    tf, hs, hi, ss, rr = oracle.tile_layout(ot, os_, oi, grain)
    S = int(ss[-1])
    assert red.count == S == api.tile_entries(gt, grain)
    # red_start per leaf: the first row of its tile's segment (tiles are runs of leaves)
    want = np.repeat(ss[:-1], np.diff(tf))
    got = _n(red.red_start)
    np.testing.assert_array_equal(got[:gt.n_leaves], want)
    assert got[gt.n_leaves] == S
    np.testing.assert_array_equal(_n(red.red_row)[:gn.count], rr)
    np.testing.assert_array_equal(_n(red.planes[0])[:S].reshape(S, -1),
                                  oracle.restructure_tile_rows(ot, hs, hi, ss, q).reshape(S, -1))


CASES = [([12, 8, 20, 4], 2), ([12, 8, 20, 4], 4), ([16], 2), ([16], 4), ([28, 4, 24], 2)]


@pytest.mark.parametrize("sides,grain", CASES)
@pytest.mark.parametrize("nrhs", [1, 3, 64])
def test_tile_layout_and_evaluation(sides, grain, nrhs):
    print(f"case tiles sides={sides} grain={grain} nrhs={nrhs}", flush=True)
    gt, gn = _tree(sides)
    q = W.grid_rhs(gt.n, nrhs, seed=51)
    if nrhs == 1:
        q = q[:, 0].copy()
    ref = oracle.helmholtz(sides, q)
    precs = [("fp32", np.complex64, TOL32)] + ([("fp64", np.complex128, TOL64)] if nrhs < 64 else [])
    for prec, cd, tol in precs:
        qc = q.astype(cd)
        gq = torch.as_tensor(qc, device=DEV)
        red = api.restructure(gt, gn, [gq], prec=prec, nrhs=nrhs, grain=grain)
        _check_layout(gt, gn, red, sides, grain, qc)
        u = _n(api.helmholtz(gt, gn, None, layout="redundant", prec=prec, red=red, nrhs=nrhs))
        box = api.restructure(gt, gn, [gq], prec=prec, nrhs=nrhs)
        ub = _n(api.helmholtz(gt, gn, None, layout="redundant", prec=prec, red=box, nrhs=nrhs))
        err = _rel(u, ref)
        print(f"  {prec}: {err:.2e}", flush=True)
        assert err <= tol
        # the same sums in the same order as the box-grain layout: the same bits
        np.testing.assert_array_equal(u, ub)


def test_tile_layout_twice_into_one_buffer_and_capacity():
    """A second restructure into the same buffers gives the same bits as the
    first; a too-small buffer is refused with P2P_ECAPACITY."""
    sides = [20, 12]
    gt, gn = _tree(sides)
    q = torch.as_tensor(W.grid_rhs(gt.n, 64, seed=52), device=DEV)
    red4 = api.restructure(gt, gn, [q], prec="fp32", nrhs=64, grain=4)
    first = _n(red4.planes[0])[:red4.count].copy()
    api.restructure(gt, gn, [q], prec="fp32", nrhs=64, out=red4)
    np.testing.assert_array_equal(_n(red4.planes[0])[:red4.count], first)
    small = api.Redundant(count=0, red_start=torch.empty(gt.n_leaves + 1, dtype=torch.int64, device=DEV),
                          red_self=torch.empty(gt.n_leaves, dtype=torch.int32, device=DEV),
                          planes=[torch.empty((64, 64), dtype=torch.complex64, device=DEV), None, None, None],
                          nrhs=64, kind=1, prec=1, grain=2,
                          red_row=torch.empty(gn.count, dtype=torch.int64, device=DEV))
    with pytest.raises(api.L.P2PError) as ei:
        api.restructure(gt, gn, [q], prec="fp32", nrhs=64, out=small)
    assert ei.value.status == api.L.P2P_ECAPACITY

"""Helmholtz batches whose instances differ in k h (several tables of G
blocks or G(dd) values, each instance reading its own) and single-RHS
matrix-core batches of more than 8 instances (parameters uploaded instead of
passed in the kernel arguments), against the FP64 oracle with each instance's
own h and k, in both layouts and precisions."""
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


def _batch(sides, ppw, span):
    """Instances of edge n with spacing span/n and k for `ppw` points per
    wavelength: k h = 2 pi / ppw differs between instances with different ppw."""
    h = np.array([s / n for n, s in zip(sides, span)], dtype=np.float64)
    kw = np.array([2 * np.pi / (p * hh) for p, hh in zip(ppw, h)], dtype=np.float64)
    grids = [api.Grid(int(n), float(hh), float(k)) for n, hh, k in zip(sides, h, kw)]
    return grids, h, kw


def _check(sides, ppw, span, nrhs, seed, precs):
    grids, h, kw = _batch(sides, ppw, span)
    gt = api.Tree.build_grids(grids, device=DEV)
    gn = gt.neighbors()
    q = W.grid_rhs(gt.n, nrhs, seed=seed)
    if nrhs == 1:
        q = q[:, 0].copy()
    ref = oracle.helmholtz(sides, q, h=h, kw=kw)
    errs = {}
    for prec, cd, tol in precs:
        gq = torch.as_tensor(q.astype(cd), device=DEV)
        red = api.restructure(gt, gn, [gq], prec=prec, nrhs=nrhs)
        for layout in ("gather", "redundant"):
            u = _n(api.helmholtz(gt, gn, gq, layout=layout, prec=prec, red=red, nrhs=nrhs))
            err = _rel(u, ref)
            # each instance on its own as well: a wrong table shows in its instance
            off = np.concatenate([[0], np.cumsum(np.asarray(sides, dtype=np.int64) ** 3)])
            per = [_rel(u[off[i]:off[i + 1]], ref[off[i]:off[i + 1]]) for i in range(len(sides))]
            print(f"  {prec} {layout}: {err:.2e}, worst instance {max(per):.2e}", flush=True)
            assert err <= tol and max(per) <= tol, (prec, layout, per)
            errs[(prec, layout)] = err
    return errs


FP32 = ("fp32", np.complex64, TOL32)
FP64 = ("fp64", np.complex128, TOL64)


@pytest.mark.parametrize("nrhs", [1, 3, 64])
def test_instances_with_different_kh(nrhs):
    """Four instances, three distinct k h (10, 6 and 14 points per wavelength)
    and spacings that are not all 1/n: three G tables."""
    sides, ppw, span = [16, 12, 20, 8], [10, 6, 10, 14], [1.0, 0.75, 1.0, 2.0]
    print(f"case kh tables sides={sides} ppw={ppw} nrhs={nrhs}", flush=True)
    _check(sides, ppw, span, nrhs, 31, [FP32, FP64] if nrhs < 64 else [FP32])


def test_multi_rhs_tables_with_tiles():
    """The multi-RHS matrix-core path with several tables under every copy count
    of the G blocks and both RHS tiles: the same results."""
    sides, ppw, span = [12, 16, 8], [6, 10, 20], [1.0, 1.0, 0.5]
    grids, h, kw = _batch(sides, ppw, span)
    gt = api.Tree.build_grids(grids, device=DEV)
    gn = gt.neighbors()
    q = W.grid_rhs(gt.n, 64, seed=32)
    ref = oracle.helmholtz(sides, q, h=h, kw=kw)
    gq = torch.as_tensor(q, device=DEV)
    base = None
    for tile in ((4, 2, 64, 1), (4, 2, 32, 2), (2, 4, 64, 4), (1, 8, 32, 8)):
        print(f"case tables tile={tile}", flush=True)
        u = _n(api.helmholtz(gt, gn, gq, prec="fp32", tile=tile))
        assert _rel(u, ref) <= TOL32
        if base is None:
            base = u
        elif tile[2] == 64:
            np.testing.assert_array_equal(u, base)


@pytest.mark.parametrize("n_inst,mixed_kh", [(9, False), (12, True)])
def test_single_rhs_matrix_cores_many_instances(n_inst, mixed_kh):
    """Single right-hand side on the matrix cores with more than 8 instances,
    whose parameters (tiles, tables, 1/h) are uploaded; one table or several."""
    rng = np.random.default_rng(33 + n_inst)
    sides = [int(4 * v) for v in rng.integers(1, 6, n_inst)]
    ppw = [10 if not mixed_kh else [10, 6, 14][i % 3] for i in range(n_inst)]
    span = [1.0] * n_inst
    print(f"case single-RHS {n_inst} instances sides={sides} ppw={ppw}", flush=True)
    _check(sides, ppw, span, 1, 34, [FP32, FP64])

"""The two single-precision Helmholtz modes against the FP64 oracle: FP32_MIXED
(each near box's FP32 partial product added into FP64 per-target sums) and
FP32 (single precision throughout), on every evaluation path (single RHS and
multiple of 32 RHS on the matrix cores, ragged RHS counts on the vector
units), both layouts; a layout built in one mode serves the other."""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_21535_amd import api
from paper_2511_21535_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
DEV = "cuda"


def _rel(a, b):
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("sides,nrhs", [([24, 16], 1), ([24, 16], 3), ([24, 16], 64), ([32], 32)])
def test_single_precision_modes(sides, nrhs):
    print(f"case precision modes sides={sides} nrhs={nrhs}", flush=True)
    grids = [api.Grid(int(s), *W.grid_geometry(int(s))) for s in sides]
    gt = api.Tree.build_grids(grids, device=DEV)
    gn = gt.neighbors()
    q = W.grid_rhs(gt.n, nrhs, seed=61)
    if nrhs == 1:
        q = q[:, 0].copy()
    ref = oracle.helmholtz(sides, q)
    gq = torch.as_tensor(q, device=DEV)
    red_plain = api.restructure(gt, gn, [gq], prec="fp32_plain", nrhs=nrhs)
    red_mixed = api.restructure(gt, gn, [gq], prec="fp32", nrhs=nrhs)
    np.testing.assert_array_equal(red_plain.planes[0].cpu().numpy(), red_mixed.planes[0].cpu().numpy())
    errs = {}
    for prec in ("fp32", "fp32_plain"):
        outs = []
        for layout, red in (("gather", None), ("redundant", red_mixed), ("redundant", red_plain)):
            u = api.helmholtz(gt, gn, gq if red is None else None, layout=layout, prec=prec, red=red,
                              nrhs=nrhs).cpu().numpy()
            outs.append(u)
            err = _rel(u, ref)
            per = max(_rel(u.reshape(gt.n, -1)[:, j], ref.reshape(gt.n, -1)[:, j]) for j in range(nrhs))
            assert err <= TOL32 and per <= TOL32, (prec, layout, err, per)
        # the layouts give the same sums in the same order
        np.testing.assert_array_equal(outs[1], outs[2])
        errs[prec] = _rel(outs[0], ref)
    print(f"  rel L2: FP32_MIXED {errs['fp32']:.2e}, FP32 {errs['fp32_plain']:.2e}", flush=True)


def test_adjoint_in_both_single_precision_modes():
    sides = [20]
    grids = [api.Grid(20, *W.grid_geometry(20))]
    gt = api.Tree.build_grids(grids, device=DEV)
    gn = gt.neighbors()
    g = W.grid_rhs(gt.n, 1, seed=62)[:, 0].copy()
    ref = oracle.helmholtz_transpose(sides, g)
    for prec in ("fp32", "fp32_plain"):
        got = api.helmholtz_adjoint(gt, gn, torch.as_tensor(g, device=DEV), prec=prec).cpu().numpy()
        assert _rel(got, ref) <= TOL32, prec

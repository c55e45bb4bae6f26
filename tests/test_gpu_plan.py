"""Helmholtz evaluation from a plan (p2p_helmholtz_prepare once, then
p2p_eval_helmholtz_prepared): bit for bit the results of p2p_eval_helmholtz,
which builds the same set-up on every call, on every path -- single RHS on
the matrix cores in FP32 and FP64 with parameters in the kernel arguments and
uploaded (more than 8 instances), several tables of G blocks, multi-RHS on the
matrix cores with and without a tile, the vector kernel in FP32 and FP64 -- in both
layouts and both grains, repeated calls from one plan, and within the
tolerances of the FP64 oracle."""
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


def _grids(sides, ppw):
    h = np.array([1.0 / n for n in sides], dtype=np.float64)
    kw = np.array([2 * np.pi / (p * hh) for p, hh in zip(ppw, h)], dtype=np.float64)
    return [api.Grid(int(n), float(hh), float(k)) for n, hh, k in zip(sides, h, kw)], h, kw


CASES = [
    # sides, points per wavelength, nrhs, prec, tile
    ([16], [10], 1, "fp32", None),
    ([16], [10], 1, "fp32_plain", None),
    ([12, 8, 20, 4], [10, 6, 10, 8], 1, "fp32", None),
    ([8] * 5 + [4] * 5, [10, 6] * 5, 1, "fp32", None),          # 10 instances: parameters uploaded
    ([12, 8], [10, 6], 64, "fp32", None),
    ([12, 8], [10, 6], 64, "fp32", (4, 2, 32, 2)),
    ([12, 8], [10, 10], 3, "fp32", None),
    ([12, 8], [10, 6], 3, "fp64", None),
    ([12, 8, 20, 4], [10, 6, 10, 8], 1, "fp64", None),        # FP64 matrix cores, tiles split in two
    ([8] * 5 + [4] * 5, [10, 6] * 5, 1, "fp64", None),        # ... with uploaded parameters (1/h in double)
]


@pytest.mark.parametrize("sides,ppw,nrhs,prec,tile", CASES)
def test_prepared_equals_per_call(sides, ppw, nrhs, prec, tile):
    print(f"case plan sides={sides} nrhs={nrhs} prec={prec} tile={tile}", flush=True)
    grids, h, kw = _grids(sides, ppw)
    gt = api.Tree.build_grids(grids, device=DEV)
    gn = gt.neighbors()
    q = W.grid_rhs(gt.n, nrhs, seed=61)
    if nrhs == 1:
        q = q[:, 0].copy()
    cd = np.complex128 if prec == "fp64" else np.complex64
    gq = torch.as_tensor(q.astype(cd), device=DEV)
    ref = oracle.helmholtz(sides, q, h=h, kw=kw)
    tol = TOL64 if prec == "fp64" else TOL32
    plan = api.HelmholtzPlan(gt, gn, prec=prec, nrhs=nrhs, tile=tile)
    for grain in (0, 2):
        red = api.restructure(gt, gn, [gq], prec=prec, nrhs=nrhs, grain=grain)
        for layout in ("gather", "redundant"):
            want = _n(api.helmholtz(gt, gn, gq, layout=layout, prec=prec, red=red, nrhs=nrhs, tile=tile))
            for _ in range(2):
                got = _n(api.helmholtz(gt, gn, gq, layout=layout, red=red, plan=plan))
                np.testing.assert_array_equal(got, want)
            err = _rel(got, ref)
            print(f"  grain {grain} {layout}: {err:.2e}", flush=True)
            assert err <= tol


def test_prepared_refuses_other_arguments():
    grids, _, _ = _grids([12, 8], [10, 6])
    gt = api.Tree.build_grids(grids, device=DEV)
    gn = gt.neighbors()
    plan = api.HelmholtzPlan(gt, gn, prec="fp32", nrhs=1)
    other, _, _ = _grids([12, 8], [10, 7])
    ot = api.Tree.build_grids(other, device=DEV)
    on = ot.neighbors()
    q = torch.as_tensor(W.grid_rhs(gt.n, 1, seed=62)[:, 0].astype(np.complex64), device=DEV)
    with pytest.raises(api.L.P2PError) as ei:
        api.helmholtz(ot, on, q, plan=plan)
    assert ei.value.status == api.L.P2P_EINVAL and "prepared for another" in str(ei.value)

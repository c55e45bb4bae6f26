"""GPU parity of the multi-RHS matrix-core Helmholtz path, the batched
persistent launch, the autotuner, the autograd wrappers and the adjoint
workloads, against the FP64 oracle (FP32 paths <= 1e-5, FP64 <= 1e-12)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2511_21535_amd import api, autograd, autotune
from paper_2511_21535_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL32, TOL64 = 1e-5, 1e-12


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def _n(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _grid_tree(sides):
    grids = [api.Grid(int(n), *W.grid_geometry(int(n))) for n in sides]
    t = api.Tree.build_grids(grids)
    return t, t.neighbors()


# [4] and [4, 8]: one and nine boxes, fewer (box, RHS chunk) items than the
# product's eight per-XCD queues, most of which start empty
@pytest.mark.parametrize("sides,nrhs", [([16], 64), ([12, 8, 20], 32), ([8, 16], 96), ([4], 32), ([4, 8], 64)])
def test_helmholtz_mfma_parity(sides, nrhs):
    print(f"case mfma sides={sides} nrhs={nrhs}", flush=True)
    gt, gn = _grid_tree(sides)
    q = W.grid_rhs(gt.n, nrhs, seed=61)
    ref = oracle.helmholtz(sides, q)
    gq = _t(q)
    red = api.restructure(gt, gn, [gq], prec="fp32", nrhs=nrhs)
    # payload bit-exact (rows of 8 nrhs bytes in 16-byte units)
    ot = oracle.build_tree_grids(sides)
    os_, oi = oracle.neighbors(ot)
    rs, _, S = oracle.red_offsets(ot, os_, oi)
    assert red.count == S
    np.testing.assert_array_equal(_n(red.planes[0])[:S], oracle.restructure_rows(ot, os_, oi, rs, q))
    for layout in ("gather", "redundant"):
        u = _n(api.helmholtz(gt, gn, gq, layout=layout, prec="fp32", red=red))
        err = _rel(u, ref)
        # per-column errors too: every right-hand side must meet the bar
        col = max(_rel(u[:, r], ref[:, r]) for r in range(nrhs))
        print(f"  {layout}: {err:.2e} (worst column {col:.2e})", flush=True)
        assert err <= TOL32 and col <= TOL32


def test_mfma_tiles_agree_and_conjugate():
    gt, gn = _grid_tree([12, 16])
    q = W.grid_rhs(gt.n, 64, seed=62)
    gq = _t(q)
    # FP32_MIXED: 32 right-hand sides per wave take the complex product as three real
    # products, 64 per wave (with the FP64 sums) as four; within one product form every
    # launch shape and every number of copies of the G blocks gives the same bits, and
    # the two forms agree with each other and with the oracle
    base = {r: _n(api.helmholtz(gt, gn, gq, prec="fp32", tile=(4, 2, r, 1))) for r in (32, 64)}
    for tile in list(autotune.CANDIDATES) + [(4, 2, 64, c) for c in autotune.COPIES]:
        u = _n(api.helmholtz(gt, gn, gq, prec="fp32", tile=tile))
        np.testing.assert_array_equal(u, base[tile[2]])
    ref = oracle.helmholtz([12, 16], q)
    assert _rel(base[32], base[64]) <= 1e-6
    assert _rel(base[32], ref) <= TOL32 and _rel(base[64], ref) <= TOL32
    # conjugated action A^H g = conj(A conj(g)) on the matrix cores
    outc = _n(api.helmholtz_adjoint(gt, gn, gq, prec="fp32", conjugate=True))
    assert _rel(outc, np.conj(oracle.helmholtz([12, 16], np.conj(q)))) <= TOL32


def test_batched_equals_singles():
    sides = [12, 8, 20, 16]
    gt, gn = _grid_tree(sides)
    q = W.grid_rhs(gt.n, 32, seed=63)
    ub = _n(api.helmholtz(gt, gn, _t(q), prec="fp32"))
    off = oracle.grid_offsets(sides)
    for g, n in enumerate(sides):
        t1, n1 = _grid_tree([n])
        u1 = _n(api.helmholtz(t1, n1, _t(q[off[g]:off[g + 1]]), prec="fp32"))
        assert _rel(ub[off[g]:off[g + 1]], u1) <= 1e-6


@pytest.mark.slow
def test_full_batched_128x64_sampled():
    """128 grids of edge 16..48, 64 right-hand sides, one persistent launch,
    both layouts, autotuned tile; sampled targets against the oracle."""
    w = W.WORKLOADS["helmholtz_batched_128x64"]
    sides = W.batched_grid_sides(w["n_instances"], w["seed"])
    print(f"case batched: {len(sides)} grids, {int((sides.astype(np.int64) ** 3).sum())} points", flush=True)
    gt, gn = _grid_tree(sides)
    q = W.grid_rhs(gt.n, w["nrhs"], seed=w["seed"])
    gq = _t(q)
    rng = np.random.default_rng(2)
    tg = np.unique(np.concatenate([rng.choice(gt.n, 300, replace=False), [0, gt.n - 1]]))
    ref = oracle.helmholtz(sides, q, targets=tg)
    tile, ms = autotune.tune_helmholtz(gt, gn, q=gq, layout="gather", use_cache=False)
    print(f"  autotuned tile {tile}: {min(ms.values()):.2f} ms", flush=True)
    u = _n(api.helmholtz(gt, gn, gq, prec="fp32", tile=tile)[torch.as_tensor(tg, device=DEV)])
    err = _rel(u, ref)
    print(f"  gather: {err:.2e}", flush=True)
    assert err <= TOL32
    del u
    red = api.restructure(gt, gn, [gq], prec="fp32", nrhs=w["nrhs"])
    u = _n(api.helmholtz(gt, gn, None, layout="redundant", prec="fp32", red=red,
                         tile=tile)[torch.as_tensor(tg, device=DEV)])
    err = _rel(u, ref)
    print(f"  redundant: {err:.2e} (S = {red.count})", flush=True)
    assert err <= TOL32
    loc = api.locality(gt, gn, red)
    assert loc["entries"] == red.count


# ------------------------------------------------------------ autograd
def test_gravity_gradcheck():
    x, y, z, m = W.plummer_mixture(40, 71)
    t = [torch.tensor(v, device=DEV, dtype=torch.float64, requires_grad=True) for v in (x, y, z, m)]
    tree = api.Tree.build_particles(*[v.detach() for v in t[:3]], depth=20, leaf_cap=8)
    nbrs = tree.neighbors()
    f = lambda a, b, c, d: autograd.gravity(a, b, c, d, tree, nbrs, 2e-2)
    assert torch.autograd.gradcheck(f, tuple(t), eps=1e-7, atol=1e-6, rtol=1e-5)


def test_helmholtz_gradcheck_and_contrast():
    gt, gn = _grid_tree([8])
    q = torch.tensor(W.grid_rhs(gt.n, 1, seed=72)[:, 0].astype(np.complex128), device=DEV,
                     requires_grad=True)
    f = lambda v: autograd.helmholtz(v, gt, gn, "fp64")
    assert torch.autograd.gradcheck(f, (q,), eps=1e-7, atol=1e-7, rtol=1e-5)
    # contrast chi (real), q = chi * u_inc: dL/dchi = Re(conj(u_inc) * dL/dq)
    uinc = torch.tensor(W.grid_rhs(gt.n, 1, seed=73)[:, 0].astype(np.complex128), device=DEV)
    chi = torch.rand(gt.n, dtype=torch.float64, device=DEV, requires_grad=True)
    f2 = lambda c: autograd.helmholtz(c * uinc, gt, gn, "fp64")
    assert torch.autograd.gradcheck(f2, (chi,), eps=1e-7, atol=1e-7, rtol=1e-5)


# ------------------------------------------------------------ adjoint workloads
@pytest.mark.slow
def test_adjoint_gravity_256k():
    """2^18 Plummer particles, cap 64, FP64: the adjoint against the oracle's on
    sampled leaves, and central differences (h = 1e-6, tree frozen) of the GPU
    forward on 16 sampled coordinates."""
    w = W.WORKLOADS["adjoint_gravity_256k"]
    x, y, z, m = W.particles("adjoint_gravity_256k")
    n = len(x)
    gp, gax, gay, gaz = (W.normal_like(n, seed=w["seed"] + 10 * k) for k in range(1, 5))
    gx_, gy_, gz_, gm_ = (_t(v) for v in (x, y, z, m))
    gg = [_t(v) for v in (gp, gax, gay, gaz)]
    tree = api.Tree.build_particles(gx_, gy_, gz_, depth=w["depth"], leaf_cap=w["leaf_cap"])
    nbrs = tree.neighbors()
    adj = [_n(v) for v in api.gravity_adjoint(tree, nbrs, w["eps"], gx_, gy_, gz_, gm_, *gg)]
    ot = oracle.build_tree_particles(x, y, z, depth=w["depth"], leaf_cap=w["leaf_cap"])
    rng = np.random.default_rng(5)
    sel = np.sort(rng.choice(ot.n_leaves, 64, replace=False)).astype(np.int32)
    ss, si = oracle.neighbors(ot, sel)
    idx, rm, rx, ry, rz = oracle.gravity_adjoint_leaves(x, y, z, m, w["eps"], gp, gax, gay, gaz, ot,
                                                        sel, ss, si)
    assert _rel(adj[3][idx], rm) <= TOL64
    assert _rel(np.stack([a[idx] for a in adj[:3]]), np.stack([rx, ry, rz])) <= TOL64
    # the FP32-mixed adjoint against the same oracle values
    adj32 = [_n(v) for v in api.gravity_adjoint(tree, nbrs, w["eps"], gx_, gy_, gz_, gm_, *gg, prec="fp32")]
    assert _rel(adj32[3][idx], rm) <= TOL32
    assert _rel(np.stack([a[idx] for a in adj32[:3]]), np.stack([rx, ry, rz])) <= TOL32
    # central differences of the GPU forward; outputs untouched by the move are bitwise equal
    h = 1e-6
    scale = max(np.abs(a).max() for a in adj[:3])
    for j in rng.choice(n, 16, replace=False):
        for d, arr in enumerate((x, y, z)):
            outs = []
            for sgn in (1, -1):
                v = arr.copy()
                v[j] += sgn * h
                pos = [gx_, gy_, gz_]
                pos[d] = _t(v)
                outs.append([_n(o) for o in api.gravity(tree, nbrs, w["eps"], *pos, m=gm_)])
            diff = [a - b for a, b in zip(*outs)]
            fd = (np.dot(gp, diff[0]) + np.dot(gax, diff[1]) + np.dot(gay, diff[2])
                  + np.dot(gaz, diff[3])) / (2 * h)
            assert abs(fd - adj[d][j]) <= 1e-5 * scale, (j, d, fd, adj[d][j])


@pytest.mark.slow
def test_adjoint_helmholtz_48():
    """48^3 grid, FP64: A^T g against the oracle's transpose action, and the
    dot-product test <g, A q> = <A^T g, q>."""
    gt, gn = _grid_tree([48])
    g = W.normal_like(gt.n, seed=5, dtype=np.complex128)
    q = W.normal_like(gt.n, seed=6, dtype=np.complex128)
    out = _n(api.helmholtz_adjoint(gt, gn, _t(g), prec="fp64"))
    ref = oracle.helmholtz_transpose([48], g)
    assert _rel(out, ref) <= TOL64
    Aq = _n(api.helmholtz(gt, gn, _t(q), prec="fp64"))
    lhs, rhs = np.sum(g * Aq), np.sum(out * q)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    loc = api.locality(gt, gn)
    assert loc["pairs"] == 160878592

"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Bit-exact: tree (perm, leaf_start, leaf_key, leaf_level), near lists and the
redundant payload.  Floating point: relative L2 per result, <= 1e-12 for FP64
and <= 1e-5 for FP32 / FP32-mixed (phi; a as one 3N vector; u as one complex
N*R vector).  Full-size workloads are checked on sampled leaves, which the
oracle computes one by one.
"""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_2511_21535_amd import api
from paper_2511_21535_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
DEV = "cuda"


def _t(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV, dtype=dtype)


def _n(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _check_tree(gt, ot):
    np.testing.assert_array_equal(_n(gt.perm), ot.perm)
    # iperm is the inverse of perm
    np.testing.assert_array_equal(_n(gt.iperm)[ot.perm], np.arange(len(ot.perm), dtype=np.int32))
    np.testing.assert_array_equal(_n(gt.leaf_start), ot.leaf_start)
    np.testing.assert_array_equal(_n(gt.leaf_key).view(np.uint64), ot.leaf_key)
    np.testing.assert_array_equal(_n(gt.leaf_level), ot.leaf_level)


def _particles_case(gen, n, seed, depth, cap):
    if gen == "uniform":
        x, y, z, m = W.uniform_particles(n, seed)
    else:
        x, y, z, m = W.plummer_mixture(n, seed)
    return x, y, z, m


PARTICLE_CASES = [
    ("uniform", 4096, 1, 3, 0),       # the 4096-particle uniform depth-3 workload
    ("uniform", 3000, 7, 4, 0),
    ("plummer", 20000, 8, 20, 64),
    ("plummer", 5000, 9, 20, 8),
    ("plummer", 3001, 10, 20, 1),
    ("plummer", 777, 11, 6, 16),      # depth cap reached
    ("uniform", 20000, 13, 1, 0),     # 8 leaves of ~2500 points: segments of 20000 rows, >256 targets per leaf
    ("plummer", 30000, 14, 20, 2048),  # the largest cap of the LDS-tiled leaf levels
    ("plummer", 30000, 15, 20, 2049),  # past it: the per-slot merge over global memory
]


@pytest.mark.parametrize("gen,n,seed,depth,cap", PARTICLE_CASES)
def test_tree_neighbors_restructure_bit_exact(gen, n, seed, depth, cap):
    x, y, z, m = _particles_case(gen, n, seed, depth, cap)
    print(f"case {gen} n={n} seed={seed} depth={depth} cap={cap}", flush=True)
    gx, gy, gz, gm = (_t(v) for v in (x, y, z, m))
    gt = api.Tree.build_particles(gx, gy, gz, depth=depth, leaf_cap=cap)
    ot = oracle.build_tree_particles(x, y, z, depth=depth, leaf_cap=cap)
    _check_tree(gt, ot)
    assert gt.max_level == int(ot.leaf_level.max())
    gn = gt.neighbors()
    os_, oi = oracle.neighbors(ot)
    np.testing.assert_array_equal(_n(gn.nbr_start), os_)
    np.testing.assert_array_equal(_n(gn.nbr_idx), oi)
    rs, rself, S = oracle.red_offsets(ot, os_, oi)
    assert gn.red_entries == S
    # lists without the layout size: the restructure counts S itself
    gn_unknown = dataclasses.replace(gn, red_entries=-1)
    for prec in ("fp64", "fp32"):
        red = api.restructure_gravity(gt, gn, gx, gy, gz, gm, prec=prec)
        red_u = api.restructure_gravity(gt, gn_unknown, gx, gy, gz, gm, prec=prec)
        assert red_u.count == S
        np.testing.assert_array_equal(_n(red_u.red_start), rs)
        np.testing.assert_array_equal(_n(red_u.planes[0])[:S], _n(red.planes[0])[:S])
        assert red.count == S
        np.testing.assert_array_equal(_n(red.red_start), rs)
        np.testing.assert_array_equal(_n(red.red_self), rself)
        if prec == "fp64":
            want = oracle.restructure_rows(ot, os_, oi, rs, np.stack([x, y, z, m], 1))
            np.testing.assert_array_equal(_n(red.planes[0])[:S].view(np.uint64), want.view(np.uint64))
        else:
            want = oracle.restructure_gravity_rel(ot, os_, oi, rs, x, y, z, m)
            np.testing.assert_array_equal(_n(red.planes[0])[:S].view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("gen,n,seed,depth,cap", PARTICLE_CASES[:4] + PARTICLE_CASES[6:])
@pytest.mark.parametrize("eps_arg", [1e-3, 0.0, "min"])
def test_interaction_layout_parity(gen, n, seed, depth, cap, eps_arg):
    """Per-interaction layout: records bit-exact against the oracle, sums
    within the tolerances, with lists that carry S and lists that do not."""
    x, y, z, m = _particles_case(gen, n, seed, depth, cap)
    print(f"case interactions {gen} n={n} eps={eps_arg}", flush=True)
    gx, gy, gz, gm = (_t(v) for v in (x, y, z, m))
    gt = api.Tree.build_particles(gx, gy, gz, depth=depth, leaf_cap=cap)
    gn = gt.neighbors()
    ot = oracle.build_tree_particles(x, y, z, depth=depth, leaf_cap=cap)
    os_, oi = oracle.neighbors(ot)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32)):
        eps = EPS_MIN[prec] if eps_arg == "min" else eps_arg
        ref = oracle.gravity(x, y, z, m, eps, ot)
        rec, rows = oracle.restructure_interactions(ot, os_, oi, x, y, z, m, prec=prec)
        for lists in (gn, dataclasses.replace(gn, red_entries=-1)):
            inter = api.restructure_interactions(gt, lists, gx, gy, gz, gm, prec=prec)
            assert inter.count == len(rows)
            np.testing.assert_array_equal(_n(inter.rec_start), rec)
            got = _n(inter.rows)[:len(rows)]
            if prec == "fp64":
                np.testing.assert_array_equal(got.view(np.uint64), rows.view(np.uint64))
            else:
                np.testing.assert_array_equal(got.view(np.uint32), rows.view(np.uint32))
        o = [_n(v) for v in api.gravity_interactions(gt, gn, inter, eps)]
        e_phi, e_a = _rel(o[0], ref[0]), _rel(np.stack(o[1:]), np.stack(ref[1:]))
        print(f"  {prec}: phi {e_phi:.2e} a {e_a:.2e}", flush=True)
        assert e_phi <= tol and e_a <= tol


def test_long_near_lists():
    """Lists longer than the 64 entries the counting pass keeps per leaf."""
    x, y, z, m = W.slab_particles(4000, 16, 5e-4, seed=12)
    print("case slab 4000+16 cap 4", flush=True)
    ot = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=4)
    os_, oi = oracle.neighbors(ot)
    assert np.diff(os_).max() > 64          # the case exercises the overflow path
    gx, gy, gz, gm = (_t(v) for v in (x, y, z, m))
    gt = api.Tree.build_particles(gx, gy, gz, depth=20, leaf_cap=4)
    _check_tree(gt, ot)
    gn = gt.neighbors()
    np.testing.assert_array_equal(_n(gn.nbr_start), os_)
    np.testing.assert_array_equal(_n(gn.nbr_idx), oi)
    rs, rself, S = oracle.red_offsets(ot, os_, oi)
    assert gn.red_entries == S
    red = api.restructure_gravity(gt, gn, gx, gy, gz, gm, prec="fp32")
    np.testing.assert_array_equal(_n(red.red_start), rs)
    want = oracle.restructure_gravity_rel(ot, os_, oi, rs, x, y, z, m)
    np.testing.assert_array_equal(_n(red.planes[0])[:S].view(np.uint32), want.view(np.uint32))
    ref = oracle.gravity(x, y, z, m, 1e-3, ot)
    for layout in ("gather", "redundant"):
        o = [_n(v) for v in api.gravity(gt, gn, 1e-3, x=gx, y=gy, z=gz, m=gm, layout=layout, prec="fp32", red=red)]
        assert _rel(o[0], ref[0]) <= TOL32 and _rel(np.stack(o[1:]), np.stack(ref[1:])) <= TOL32


@pytest.mark.parametrize("periodic", [False, True])
def test_heavy_leaf_lists(periodic):
    """Large sparse leaves beside a finely split slab: thousands of candidate
    leaves for one list, which the search hands to a whole workgroup; lists,
    image codes, S and the sums against the oracle."""
    x, y, z, m = W.slab_particles(20000, 16, 5e-4, seed=12)
    print(f"case slab 20000+16 cap 4 periodic={periodic}", flush=True)
    ot = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=4)
    nb = oracle.neighbors_periodic(ot) if periodic else oracle.neighbors(ot)
    assert np.diff(nb[0]).max() > 2000
    g = [_t(v) for v in (x, y, z, m)]
    gt = api.Tree.build_particles(*g[:3], depth=20, leaf_cap=4)
    gn = gt.neighbors(periodic=periodic)
    np.testing.assert_array_equal(_n(gn.nbr_start), nb[0])
    np.testing.assert_array_equal(_n(gn.nbr_idx), nb[1])
    if periodic:
        np.testing.assert_array_equal(_n(gn.nbr_shift), nb[2])
    _, _, S = oracle.red_offsets(ot, *nb)
    assert gn.red_entries == S
    ref = oracle.gravity(x, y, z, m, 1e-3, ot, nb)
    red = api.restructure_gravity(gt, gn, *g, prec="fp32")
    for layout in ("gather", "redundant"):
        o = [_n(v) for v in api.gravity(gt, gn, 1e-3, *g, layout=layout, prec="fp32", red=red)]
        assert _rel(o[0], ref[0]) <= TOL32 and _rel(np.stack(o[1:]), np.stack(ref[1:])) <= TOL32


# a tiny softening: FP64 takes any eps with a normal square (1e-30, far below every
# pair distance here), FP32_MIXED down to 1e-4
EPS_MIN = {"fp64": 1e-30, "fp32": 1e-4}
# the FP32_MIXED adjoint's smallest accepted eps
ADJ_EPS_MIN = {"fp64": 1e-30, "fp32": 1e-3}


@pytest.mark.parametrize("gen,n,seed,depth,cap", PARTICLE_CASES[:4] + PARTICLE_CASES[6:])
@pytest.mark.parametrize("eps", [1e-3, 0.0, "min"])
def test_gravity_parity(gen, n, seed, depth, cap, eps):
    if eps == "min":
        for prec, tol in (("fp64", TOL64), ("fp32", TOL32)):
            _gravity_case(gen, n, seed, depth, cap, EPS_MIN[prec], [(prec, tol)])
    else:
        _gravity_case(gen, n, seed, depth, cap, eps, [("fp64", TOL64), ("fp32", TOL32)])


def _gravity_case(gen, n, seed, depth, cap, eps, precs):
    x, y, z, m = _particles_case(gen, n, seed, depth, cap)
    if eps == 0.0:
        # distinct points only (eps = 0 drops zero-distance pairs; the definition diverges there)
        assert len(np.unique(np.stack([x, y, z], 1), axis=0)) == n
    print(f"case {gen} n={n} eps={eps}", flush=True)
    gx, gy, gz, gm = (_t(v) for v in (x, y, z, m))
    gt = api.Tree.build_particles(gx, gy, gz, depth=depth, leaf_cap=cap)
    gn = gt.neighbors()
    ot = oracle.build_tree_particles(x, y, z, depth=depth, leaf_cap=cap)
    ref = oracle.gravity(x, y, z, m, eps, ot)
    for prec, tol in precs:
        red = api.restructure_gravity(gt, gn, gx, gy, gz, gm, prec=prec)
        for layout in ("gather", "redundant"):
            out = api.gravity(gt, gn, eps, x=gx, y=gy, z=gz, m=gm, layout=layout, prec=prec, red=red)
            o = [_n(v) for v in out]
            e_phi = _rel(o[0], ref[0])
            e_a = _rel(np.stack(o[1:]), np.stack(ref[1:]))
            print(f"  {prec} {layout}: phi {e_phi:.2e} a {e_a:.2e}", flush=True)
            assert e_phi <= tol and e_a <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_gravity_gather_equals_redundant_bitwise(prec):
    # both layouts feed the same values in the same order to every lane: identical results
    x, y, z, m = W.plummer_mixture(8000, 12)
    gx, gy, gz, gm = (_t(v) for v in (x, y, z, m))
    gt = api.Tree.build_particles(gx, gy, gz, depth=20, leaf_cap=64)
    gn = gt.neighbors()
    red = api.restructure_gravity(gt, gn, gx, gy, gz, gm, prec=prec)
    a = api.gravity(gt, gn, 1e-3, x=gx, y=gy, z=gz, m=gm, prec=prec)
    b = api.gravity(gt, gn, 1e-3, layout="redundant", red=red, prec=prec)
    c = api.gravity(gt, gn, 1e-3, layout="redundant", red=red, prec=prec)
    for u, v, w in zip(a, b, c):
        np.testing.assert_array_equal(_n(u), _n(v))
        np.testing.assert_array_equal(_n(v), _n(w))      # deterministic


def test_gravity_momentum_fp64():
    x, y, z, m = W.plummer_mixture(30000, 13)
    gx, gy, gz, gm = (_t(v) for v in (x, y, z, m))
    gt = api.Tree.build_particles(gx, gy, gz, depth=20, leaf_cap=64)
    gn = gt.neighbors()
    _, ax, ay, az = (_n(v) for v in api.gravity(gt, gn, 1e-3, x=gx, y=gy, z=gz, m=gm))
    a = np.stack([ax, ay, az], 1)
    assert np.abs((m[:, None] * a).sum(0)).max() <= 1e-13 * np.sum(m * np.linalg.norm(a, axis=1))


@pytest.mark.slow
def test_full_size_plummer_2m_sampled():
    """The 2^21-particle Plummer workload (adaptive, cap 64), FP32-mixed, in the
    benchmark's launch configuration; tree bit-exact, sampled near lists,
    payload segments and sums."""
    w = W.WORKLOADS["gravity_plummer_2m"]
    x, y, z, m = W.particles("gravity_plummer_2m")
    print("case gravity_plummer_2m: building", flush=True)
    gx, gy, gz, gm = (_t(v) for v in (x, y, z, m))
    gt = api.Tree.build_particles(gx, gy, gz, depth=w["depth"], leaf_cap=w["leaf_cap"])
    ot = oracle.build_tree_particles(x, y, z, depth=w["depth"], leaf_cap=w["leaf_cap"])
    _check_tree(gt, ot)
    gn = gt.neighbors()
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(ot.n_leaves, 96, replace=False)).astype(np.int32)
    sel[0] = 0
    sel[-1] = ot.n_leaves - 1
    ss, si = oracle.neighbors(ot, sel)
    gs, gi = _n(gn.nbr_start), _n(gn.nbr_idx)
    for k, A in enumerate(sel):
        np.testing.assert_array_equal(gi[gs[A]:gs[A + 1]], si[ss[k]:ss[k + 1]])
    red = api.restructure_gravity(gt, gn, gx, gy, gz, gm, prec="fp32")
    rs = _n(red.red_start)
    p4 = _n(red.planes[0])
    occ = np.diff(ot.leaf_start)
    for k, A in enumerate(sel[:16]):
        c = (ot.anchor[A] + 0.5 * ot.size[A]) * 2.0 ** -20
        src = np.concatenate([ot.perm[ot.leaf_start[B]:ot.leaf_start[B + 1]] for B in si[ss[k]:ss[k + 1]]])
        want = np.stack([(x[src] - c[0]).astype(np.float32), (y[src] - c[1]).astype(np.float32),
                         (z[src] - c[2]).astype(np.float32), m[src].astype(np.float32)], 1)
        np.testing.assert_array_equal(p4[rs[A]:rs[A + 1]], want)
    idx, rp, rax, ray, raz = oracle.gravity_leaves(x, y, z, m, w["eps"], ot, sel, ss, si)
    for layout in ("gather", "redundant"):
        o = [_n(v)[idx] for v in api.gravity(gt, gn, w["eps"], x=gx, y=gy, z=gz, m=gm,
                                             layout=layout, prec="fp32", red=red)]
        e_phi = _rel(o[0], rp)
        e_a = _rel(np.stack(o[1:]), np.stack([rax, ray, raz]))
        print(f"  fp32 {layout}: phi {e_phi:.2e} a {e_a:.2e}", flush=True)
        assert e_phi <= TOL32 and e_a <= TOL32
    loc = api.locality(gt, gn, red)
    assert loc["entries"] == red.count == int(occ[gi].sum())
    del red, p4
    # per-interaction layout at full size: record offsets of the sampled
    # leaves and the sampled sums
    inter = api.restructure_interactions(gt, gn, gx, gy, gz, gm, prec="fp32")
    assert inter.count == len(gi) + 2 * loc["entries"]
    rec = _n(inter.rec_start)
    lens = 1 + occ[np.repeat(np.arange(ot.n_leaves), np.diff(gs))] + occ[gi]
    np.testing.assert_array_equal(rec, np.concatenate([[0], np.cumsum(lens)]))
    o = [_n(v)[idx] for v in api.gravity_interactions(gt, gn, inter, w["eps"])]
    e_phi, e_a = _rel(o[0], rp), _rel(np.stack(o[1:]), np.stack([rax, ray, raz]))
    print(f"  fp32 per-interaction: phi {e_phi:.2e} a {e_a:.2e}", flush=True)
    assert e_phi <= TOL32 and e_a <= TOL32


# --------------------------------------------------------------- Helmholtz
def _grid_tree(sides):
    grids = [api.Grid(int(n), *W.grid_geometry(int(n))) for n in sides]
    return api.Tree.build_grids(grids), grids


@pytest.mark.parametrize("sides", [[8], [16], [20], [12, 8, 4, 16]])
def test_grid_tree_bit_exact(sides):
    gt, _ = _grid_tree(sides)
    ot = oracle.build_tree_grids(sides)
    _check_tree(gt, ot)
    gn = gt.neighbors()
    os_, oi = oracle.neighbors(ot)
    np.testing.assert_array_equal(_n(gn.nbr_start), os_)
    np.testing.assert_array_equal(_n(gn.nbr_idx), oi)
    assert gn.red_entries == oracle.red_offsets(ot, os_, oi)[2]


@pytest.mark.parametrize("sides,nrhs", [([16], 1), ([20], 1), ([12, 8, 16], 1), ([16], 3), ([12, 8], 8)])
def test_helmholtz_parity(sides, nrhs):
    print(f"case helmholtz sides={sides} nrhs={nrhs}", flush=True)
    gt, grids = _grid_tree(sides)
    gn = gt.neighbors()
    n = gt.n
    q = W.grid_rhs(n, nrhs, seed=21)
    ref = oracle.helmholtz(sides, q)
    for prec, cd, tol in (("fp32", np.complex64, TOL32), ("fp64", np.complex128, TOL64)):
        gq = _t(q.astype(cd))
        red = api.restructure(gt, gn, [gq], prec=prec, nrhs=nrhs)
        ot = oracle.build_tree_grids(sides)
        os_, oi = oracle.neighbors(ot)
        rs, rself, S = oracle.red_offsets(ot, os_, oi)
        np.testing.assert_array_equal(_n(red.red_start), rs)
        np.testing.assert_array_equal(_n(red.red_self), rself)
        np.testing.assert_array_equal(_n(red.planes[0])[:S], oracle.restructure_rows(ot, os_, oi, rs, q.astype(cd)))
        for layout in ("gather", "redundant"):
            u = _n(api.helmholtz(gt, gn, gq, layout=layout, prec=prec, red=red))
            err = _rel(u, ref)
            print(f"  {prec} {layout}: {err:.2e}", flush=True)
            assert err <= tol


@pytest.mark.parametrize("prec,tol", [("fp32", TOL32), ("fp64", TOL64)])
def test_helmholtz_full_64_sampled(prec, tol):
    """The 64^3 grid workload, both layouts; sampled targets vs the oracle.  In
    FP64 its 256 column tiles take one workgroup each (smaller grids share a
    tile's offsets between two workgroups)."""
    gt, grids = _grid_tree([64])
    gn = gt.neighbors()
    q = W.grid_rhs(gt.n, 1, seed=W.WORKLOADS["helmholtz_grid_64"]["seed"])
    gq = _t(q if prec == "fp32" else q.astype(np.complex128))
    red = api.restructure(gt, gn, [gq], prec=prec, nrhs=1)
    rng = np.random.default_rng(1)
    tg = np.unique(np.concatenate([rng.choice(gt.n, 4000, replace=False), [0, gt.n - 1]]))
    ref = oracle.helmholtz([64], q.astype(np.complex128), targets=tg)
    loc = api.locality(gt, gn, red)
    assert loc["pairs"] == 398426112
    for layout in ("gather", "redundant"):
        u = _n(api.helmholtz(gt, gn, gq, layout=layout, prec=prec, red=red))
        err = _rel(u[tg], ref)
        print(f"  64^3 {prec} {layout}: {err:.2e}", flush=True)
        assert err <= tol


# --------------------------------------------------------------- adjoint
@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("fp32", TOL32)])
@pytest.mark.parametrize("eps", [1e-3, "min"])
def test_gravity_adjoint_parity(prec, tol, eps):
    eps = ADJ_EPS_MIN[prec] if eps == "min" else eps
    print(f"case gravity adjoint {prec} eps={eps}", flush=True)
    x, y, z, m = W.plummer_mixture(3000, 31)
    gp, gax, gay, gaz = (W.normal_like(3000, seed=s) for s in (32, 33, 34, 35))
    gx, gy, gz, gm = (_t(v) for v in (x, y, z, m))
    gt = api.Tree.build_particles(gx, gy, gz, depth=20, leaf_cap=64)
    gn = gt.neighbors()
    out = [_n(v) for v in api.gravity_adjoint(gt, gn, eps, gx, gy, gz, gm, *(_t(v) for v in (gp, gax, gay, gaz)),
                                              prec=prec)]
    ot = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=64)
    rm, rx, ry, rz = oracle.gravity_adjoint(x, y, z, m, eps, gp, gax, gay, gaz, ot)
    e_m, e_x = _rel(out[3], rm), _rel(np.stack(out[:3]), np.stack([rx, ry, rz]))
    print(f"  adjoint {prec}: g_m {e_m:.2e} g_x {e_x:.2e}", flush=True)
    assert e_m <= tol and e_x <= tol


def test_helmholtz_adjoint_transpose():
    sides = [12, 8]
    gt, _ = _grid_tree(sides)
    gn = gt.neighbors()
    g = W.grid_rhs(gt.n, 1, seed=41)[:, 0].astype(np.complex128)
    ref = oracle.helmholtz_transpose(sides, g)
    out = _n(api.helmholtz_adjoint(gt, gn, _t(g), prec="fp64"))
    assert _rel(out, ref) <= TOL64
    outc = _n(api.helmholtz_adjoint(gt, gn, _t(g), prec="fp64", conjugate=True))
    assert _rel(outc, np.conj(oracle.helmholtz_transpose(sides, np.conj(g)))) <= TOL64


def test_helmholtz_single_rhs_fp32_adjoint_and_ragged_tiles():
    """One RHS in FP32 runs on the matrix cores with target boxes as columns,
    in tiles of 16 boxes that never straddle two instances: instances of 27, 8
    and 125 boxes (ragged last tiles), plain and conjugated action."""
    sides = [12, 8, 20]
    gt, _ = _grid_tree(sides)
    gn = gt.neighbors()
    g = W.grid_rhs(gt.n, 1, seed=43)[:, 0].astype(np.complex64)
    out = _n(api.helmholtz(gt, gn, _t(g), prec="fp32"))
    assert _rel(out, oracle.helmholtz(sides, g[:, None])[:, 0]) <= TOL32
    outc = _n(api.helmholtz_adjoint(gt, gn, _t(g), prec="fp32", conjugate=True))
    refc = np.conj(oracle.helmholtz_transpose(sides, np.conj(g)))
    assert _rel(outc, refc) <= TOL32


# --------------------------------------------------------------- edge cases
def test_edge_cases():
    # one particle; all particles in one leaf; duplicate points
    for pts in ([[0.5, 0.5, 0.5]], [[0.1, 0.1, 0.1]] * 5, np.random.default_rng(3).random((40, 3)) * 1e-4 + 0.3):
        P = np.asarray(pts, dtype=np.float64)
        m = np.ones(len(P))
        g = [_t(P[:, d].copy()) for d in range(3)] + [_t(m)]
        gt = api.Tree.build_particles(*g[:3], depth=20, leaf_cap=64)
        ot = oracle.build_tree_particles(P[:, 0], P[:, 1], P[:, 2], depth=20, leaf_cap=64)
        _check_tree(gt, ot)
        gn = gt.neighbors()
        ref = oracle.gravity(P[:, 0], P[:, 1], P[:, 2], m, 1e-3, ot)
        red = api.restructure_gravity(gt, gn, *g, prec="fp64")
        for layout in ("gather", "redundant"):
            out = [_n(v) for v in api.gravity(gt, gn, 1e-3, *g, layout=layout, red=red)]
            np.testing.assert_allclose(out[0], ref[0], rtol=1e-12, atol=1e-300)
    # out-of-domain coordinate: error, no launch of the later steps
    P = np.array([[0.5, 0.5, 1.0]])
    with pytest.raises(Exception, match="EDOMAIN"):
        api.Tree.build_particles(*[_t(P[:, d].copy()) for d in range(3)])
    # empty input: no leaves, empty lists and layouts, empty outputs
    e = _t(np.zeros(0))
    gt = api.Tree.build_particles(e, e, e)
    assert gt.n_leaves == 0
    gn = gt.neighbors()
    assert gn.count == 0 and gn.red_entries == 0 and _n(gn.nbr_start).tolist() == [0]
    for prec in ("fp64", "fp32"):
        red = api.restructure_gravity(gt, gn, e, e, e, e, prec=prec)
        assert red.count == 0 and _n(red.red_start).tolist() == [0]
        for layout in ("gather", "redundant"):
            out = api.gravity(gt, gn, 1e-3, e, e, e, e, layout=layout, prec=prec, red=red)
            assert all(o.numel() == 0 for o in out)


def test_locality_matches_oracle():
    x, y, z, m = W.plummer_mixture(20000, 51)
    gt = api.Tree.build_particles(_t(x), _t(y), _t(z), depth=20, leaf_cap=64)
    gn = gt.neighbors()
    ot = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=64)
    os_, oi = oracle.neighbors(ot)
    _, _, S = oracle.red_offsets(ot, os_, oi)
    v_red = S * 28.0
    # Formula (10) (the layout fits: 32 MB, and the equality edge) and Formula (11)
    # (a cache below the layout's size)
    for cache in (32 * 2 ** 20, v_red, v_red - 1.0, v_red / 4):
        loc = api.locality(gt, gn, bytes_per_entry=28.0, cache_bytes=cache)
        ref = oracle.locality(os_, oi, len(x), S, 28.0, cache)
        assert loc["entries"] == S
        assert loc["pairs"] == oracle.pair_count(ot, os_, oi)
        for k_g, k_o in (("d_mean", "D_mean"), ("v_ratio", "V_ratio"), ("locality", "locality")):
            assert abs(loc[k_g] - ref[k_o]) <= 1e-12 * abs(ref[k_o]), (cache, k_g)
    assert v_red < 32 * 2 ** 20 and ref["D_ratio"] > 2.0     # the branches give different values here


def test_capacity_errors_leave_outputs_untouched():
    """Near lists and a redundant layout given too little room: P2P_ECAPACITY
    with the required size reported, nothing written; the binding's retry
    gives the same lists."""
    import ctypes
    from paper_2511_21535_amd import _lib as L
    x, y, z, m = W.plummer_mixture(3000, 61)
    print("case capacity errors", flush=True)
    g = [_t(v) for v in (x, y, z, m)]
    gt = api.Tree.build_particles(*g[:3], depth=20, leaf_cap=16)
    ref = gt.neighbors()
    idx = torch.full((5,), -7, dtype=torch.int32, device=DEV)
    start = torch.full((gt.n_leaves + 1,), -7, dtype=torch.int64, device=DEV)
    s = L.p2p_nbrs()
    s.cap, s.nbr_start, s.nbr_idx = 5, start.data_ptr(), idx.data_ptr()
    ts = gt.struct()
    st, _ = api._call(lambda ws, nb: L.p2p_build_neighbors(ctypes.byref(ts), ctypes.byref(s), ws, nb,
                                                           api._stream()), gt.leaf_start.device)
    torch.cuda.synchronize()
    assert st == L.P2P_ECAPACITY and s.count == ref.count
    assert torch.all(idx == -7) and torch.all(start == -7)
    nb = api.build_neighbors(gt, cap=5)
    assert torch.equal(nb.nbr_idx, ref.nbr_idx) and torch.equal(nb.nbr_start, ref.nbr_start)
    S = ref.red_entries
    short = api.Redundant(count=0, red_start=torch.full((gt.n_leaves + 1,), -7, dtype=torch.int64, device=DEV),
                          red_self=torch.empty(gt.n_leaves, dtype=torch.int32, device=DEV),
                          planes=[torch.full((S - 1, 4), 3.0, dtype=torch.float64, device=DEV), None, None, None],
                          nrhs=1, kind=L.P2P_KIND_GRAVITY, prec=L.P2P_FP64)
    with pytest.raises(L.P2PError) as err:
        api.restructure_gravity(gt, ref, *g, prec="fp64", out=short)
    torch.cuda.synchronize()
    assert err.value.status == L.P2P_ECAPACITY
    assert torch.all(short.planes[0] == 3.0) and torch.all(short.red_start == -7)

"""GPU parity of the periodic near field (particles on the unit torus, the
periodic interactions of the stellar-dynamics case, Sec. 5.2) against the FP64
oracle, through the C ABI.

Bit-exact: near lists with their image codes, S, the redundant offsets and
payload (shifted rows), the per-interaction records.  Floating point: the
tolerances of the plain near field (relative L2 <= 1e-12 FP64, <= 1e-5
FP32-mixed).
"""
import numpy as np
import pytest

import oracle
from paper_2511_21535_amd import api
from paper_2511_21535_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
DEV = "cuda"


def _t(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


def _n(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(gen, n, seed):
    if gen == "uniform":
        return W.uniform_particles(n, seed)
    if gen == "slab":
        return W.slab_particles(n - 16, 16, 5e-4, seed)
    return W.plummer_mixture(n, seed)


CASES = [
    ("uniform", 4096, 1, 3, 0),      # uniform depth 3: 27 entries per leaf
    ("uniform", 20000, 13, 1, 0),    # 8 leaves: every leaf meets every leaf under several images
    ("uniform", 40, 3, 20, 64),      # one leaf (the root) meeting its own 26 images
    ("plummer", 20000, 8, 20, 64),
    ("plummer", 3001, 10, 20, 1),
    ("slab", 4016, 12, 20, 4),       # lists longer than the 64 slots of the counting pass
]


def _setup(gen, n, seed, depth, cap):
    x, y, z, m = _case(gen, n, seed)
    print(f"case periodic {gen} n={n} seed={seed} depth={depth} cap={cap}", flush=True)
    g = [_t(v) for v in (x, y, z, m)]
    gt = api.Tree.build_particles(*g[:3], depth=depth, leaf_cap=cap)
    gn = gt.neighbors(periodic=True)
    ot = oracle.build_tree_particles(x, y, z, depth=depth, leaf_cap=cap)
    return (x, y, z, m), g, gt, gn, ot


@pytest.mark.parametrize("gen,n,seed,depth,cap", CASES)
def test_periodic_lists_and_layout_bit_exact(gen, n, seed, depth, cap):
    (x, y, z, m), g, gt, gn, ot = _setup(gen, n, seed, depth, cap)
    os_, oi, osh = oracle.neighbors_periodic(ot)
    assert gn.periodic
    np.testing.assert_array_equal(_n(gn.nbr_start), os_)
    np.testing.assert_array_equal(_n(gn.nbr_idx), oi)
    np.testing.assert_array_equal(_n(gn.nbr_shift), osh)
    if gen == "slab":
        assert np.diff(os_).max() > 64
    rs, rself, S = oracle.red_offsets(ot, os_, oi, osh)
    assert gn.red_entries == S
    for prec in ("fp64", "fp32"):
        red = api.restructure_gravity(gt, gn, *g, prec=prec)
        assert red.count == S
        np.testing.assert_array_equal(_n(red.red_start), rs)
        np.testing.assert_array_equal(_n(red.red_self), rself)
        got = _n(red.planes[0])[:S]
        if prec == "fp64":
            want = oracle.restructure_gravity_rows(ot, os_, oi, rs, x, y, z, m, osh)
            np.testing.assert_array_equal(got.view(np.uint64), want.view(np.uint64))
        else:
            want = oracle.restructure_gravity_rel(ot, os_, oi, rs, x, y, z, m, osh)
            np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("gen,n,seed,depth,cap", CASES)
@pytest.mark.parametrize("eps", [1e-3, 0.0])
def test_periodic_gravity_parity(gen, n, seed, depth, cap, eps):
    (x, y, z, m), g, gt, gn, ot = _setup(gen, n, seed, depth, cap)
    nb = oracle.neighbors_periodic(ot)
    ref = oracle.gravity(x, y, z, m, eps, ot, nb)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32)):
        red = api.restructure_gravity(gt, gn, *g, prec=prec)
        for layout in ("gather", "redundant"):
            o = [_n(v) for v in api.gravity(gt, gn, eps, *g, layout=layout, prec=prec, red=red)]
            e_phi, e_a = _rel(o[0], ref[0]), _rel(np.stack(o[1:]), np.stack(ref[1:]))
            print(f"  {prec} {layout}: phi {e_phi:.2e} a {e_a:.2e}", flush=True)
            assert e_phi <= tol and e_a <= tol
        # per-interaction layout: records bit-exact, sums within the tolerance
        rec, rows = oracle.restructure_interactions(ot, nb[0], nb[1], x, y, z, m, prec=prec,
                                                    nbr_shift=nb[2])
        inter = api.restructure_interactions(gt, gn, *g, prec=prec)
        np.testing.assert_array_equal(_n(inter.rec_start), rec)
        view = np.uint64 if prec == "fp64" else np.uint32
        np.testing.assert_array_equal(_n(inter.rows)[:len(rows)].view(view), rows.view(view))
        o = [_n(v) for v in api.gravity_interactions(gt, gn, inter, eps)]
        e_phi, e_a = _rel(o[0], ref[0]), _rel(np.stack(o[1:]), np.stack(ref[1:]))
        print(f"  {prec} per-interaction: phi {e_phi:.2e} a {e_a:.2e}", flush=True)
        assert e_phi <= tol and e_a <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_periodic_gather_equals_redundant_bitwise(prec):
    x, y, z, m = W.plummer_mixture(8000, 12)
    g = [_t(v) for v in (x, y, z, m)]
    gt = api.Tree.build_particles(*g[:3], depth=20, leaf_cap=64)
    gn = gt.neighbors(periodic=True)
    red = api.restructure_gravity(gt, gn, *g, prec=prec)
    a = api.gravity(gt, gn, 1e-3, *g, prec=prec)
    b = api.gravity(gt, gn, 1e-3, layout="redundant", red=red, prec=prec)
    for u, v in zip(a, b):
        np.testing.assert_array_equal(_n(u), _n(v))


@pytest.mark.parametrize("prec,tol", [("fp64", TOL64), ("fp32", TOL32)])
def test_periodic_adjoint_parity(prec, tol):
    x, y, z, m = W.plummer_mixture(3000, 31)
    gp, gax, gay, gaz = (W.normal_like(3000, seed=s) for s in (32, 33, 34, 35))
    g = [_t(v) for v in (x, y, z, m)]
    gt = api.Tree.build_particles(*g[:3], depth=20, leaf_cap=64)
    gn = gt.neighbors(periodic=True)
    out = [_n(v) for v in api.gravity_adjoint(gt, gn, 1e-3, *g, *(_t(v) for v in (gp, gax, gay, gaz)),
                                              prec=prec)]
    ot = oracle.build_tree_particles(x, y, z, depth=20, leaf_cap=64)
    rm, rx, ry, rz = oracle.gravity_adjoint(x, y, z, m, 1e-3, gp, gax, gay, gaz, ot,
                                            oracle.neighbors_periodic(ot))
    assert _rel(out[3], rm) <= tol
    assert _rel(np.stack(out[:3]), np.stack([rx, ry, rz])) <= tol


@pytest.mark.slow
def test_periodic_full_size_plummer_2m_sampled():
    """The 2^21-particle Plummer workload on the torus, FP32-mixed, in the
    benchmark's launch configuration: sampled lists, payload segments and sums."""
    w = W.WORKLOADS["gravity_plummer_2m"]
    x, y, z, m = W.particles("gravity_plummer_2m")
    print("case periodic gravity_plummer_2m: building", flush=True)
    g = [_t(v) for v in (x, y, z, m)]
    gt = api.Tree.build_particles(*g[:3], depth=w["depth"], leaf_cap=w["leaf_cap"])
    ot = oracle.build_tree_particles(x, y, z, depth=w["depth"], leaf_cap=w["leaf_cap"])
    np.testing.assert_array_equal(_n(gt.leaf_start), ot.leaf_start)
    gn = gt.neighbors(periodic=True)
    # sampled leaves, the domain's first and last among them (both touch faces)
    rng = np.random.default_rng(0)
    sel = np.sort(rng.choice(ot.n_leaves, 96, replace=False)).astype(np.int32)
    sel[0], sel[-1] = 0, ot.n_leaves - 1
    ss, si, ssh = oracle.neighbors_periodic(ot, sel)
    assert np.any(ssh != 13)
    gs, gi, gsh = _n(gn.nbr_start), _n(gn.nbr_idx), _n(gn.nbr_shift)
    for k, A in enumerate(sel):
        np.testing.assert_array_equal(gi[gs[A]:gs[A + 1]], si[ss[k]:ss[k + 1]])
        np.testing.assert_array_equal(gsh[gs[A]:gs[A + 1]], ssh[ss[k]:ss[k + 1]])
    red = api.restructure_gravity(gt, gn, *g, prec="fp32")
    rs = _n(red.red_start)
    p4 = _n(red.planes[0])
    shift = oracle.shift_vectors(ssh)
    for k, A in enumerate(sel[:16]):
        c = (ot.anchor[A] + 0.5 * ot.size[A]) * 2.0 ** -20
        parts = []
        for e in range(ss[k], ss[k + 1]):
            j = ot.perm[ot.leaf_start[si[e]]:ot.leaf_start[si[e] + 1]]
            parts.append(np.stack([((x[j] + shift[e, 0]) - c[0]).astype(np.float32),
                                   ((y[j] + shift[e, 1]) - c[1]).astype(np.float32),
                                   ((z[j] + shift[e, 2]) - c[2]).astype(np.float32),
                                   m[j].astype(np.float32)], 1))
        np.testing.assert_array_equal(p4[rs[A]:rs[A + 1]], np.concatenate(parts))
    idx, rp, rax, ray, raz = oracle.gravity_leaves(x, y, z, m, w["eps"], ot, sel, ss, si, ssh)
    for layout in ("gather", "redundant"):
        o = [_n(v)[idx] for v in api.gravity(gt, gn, w["eps"], *g, layout=layout, prec="fp32", red=red)]
        e_phi, e_a = _rel(o[0], rp), _rel(np.stack(o[1:]), np.stack([rax, ray, raz]))
        print(f"  fp32 {layout}: phi {e_phi:.2e} a {e_a:.2e}", flush=True)
        assert e_phi <= TOL32 and e_a <= TOL32

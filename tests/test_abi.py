"""C ABI checks that need no GPU: the library loads, exports every entry
point include/p2p.h declares, sizes workspaces, and rejects bad arguments on
the host before any launch."""
import ctypes
import os
import re

import pytest

from paper_2511_21535_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "p2p.h")).read()
    return sorted(set(re.findall(r"^\S.*?\b(p2p_[a-z_]+)\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2511_21535_amd import build
        build.build()
    return L.load()


def test_exports_every_declared_symbol(lib):
    decl = _declared()
    assert set(decl) >= {"p2p_build_tree", "p2p_build_neighbors", "p2p_restructure_redundant",
                         "p2p_eval_gravity", "p2p_eval_helmholtz", "p2p_adjoint"}
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(L.EXPORTED)
    # the binding offers every entry point under its C name
    for name in L.EXPORTED:
        assert callable(getattr(L, name, None)), name
    assert "gfx950" in L.p2p_version()


def _tree(n, kind=L.P2P_TREE_PARTICLES, L_=0):
    t = L.p2p_tree()
    t.n, t.cap_leaves, t.n_leaves, t.kind, t.key_bits = n, n, L_, kind, 20
    return t


def test_workspace_query_needs_no_device(lib):
    t = _tree(1000)
    nb = ctypes.c_size_t(0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: only the size is asked for
    st = lib.p2p_build_tree(fake, fake, fake, None, 0, 20, 64, ctypes.byref(t), None,
                            ctypes.byref(nb), None)
    assert st == L.P2P_OK and nb.value > 1000 * 8


@pytest.mark.parametrize("depth,cap,n_grids", [(21, 64, 0), (-1, 0, 0), (20, -1, 0), (20, 64, 2)])
def test_build_tree_rejects_bad_arguments(lib, depth, cap, n_grids):
    t = _tree(10)
    nb = ctypes.c_size_t(0)
    fake = ctypes.c_void_p(0x1000)
    st = lib.p2p_build_tree(fake, fake, fake, None, n_grids, depth, cap, ctypes.byref(t), None,
                            ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL
    assert L.last_error()


def test_build_tree_rejects_bad_grids(lib):
    g = (L.p2p_grid * 2)()
    g[0].n_side, g[0].h, g[0].k, g[0].point_off = 16, 1 / 16, 1.0, 0
    g[1].n_side, g[1].h, g[1].k, g[1].point_off = 18, 1 / 18, 1.0, 16 ** 3   # not a multiple of 4
    t = _tree(16 ** 3 + 18 ** 3, L.P2P_TREE_GRIDS)
    nb = ctypes.c_size_t(0)
    st = lib.p2p_build_tree(None, None, None, g, 2, 0, 0, ctypes.byref(t), None, ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "multiple of 4" in L.last_error()
    g[1].n_side = 20
    st = lib.p2p_build_tree(None, None, None, g, 2, 0, 0, ctypes.byref(t), None, ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "!= tree->n" in L.last_error()
    t.n = 16 ** 3 + 20 ** 3
    st = lib.p2p_build_tree(None, None, None, g, 2, 0, 0, ctypes.byref(t), None, ctypes.byref(nb), None)
    assert st == L.P2P_OK


def test_eval_rejects_bad_modes(lib):
    t = _tree(10, L_=1)
    t.perm = t.iperm = t.leaf_start = t.leaf_key = t.leaf_level = 0x1000
    n = L.p2p_nbrs()
    n.count, n.nbr_start, n.nbr_idx = 1, 0x1000, 0x1000
    nb = ctypes.c_size_t(0)
    z = ctypes.c_void_p(0x1000)
    args = lambda layout, prec, eps: (ctypes.byref(t), ctypes.byref(n), None, layout, prec, eps,
                                      z, z, z, z, z, z, z, z, None, ctypes.byref(nb), None)
    assert lib.p2p_eval_gravity(*args(7, L.P2P_FP64, 1e-3)) == L.P2P_EINVAL
    assert lib.p2p_eval_gravity(*args(L.P2P_GATHER, 9, 1e-3)) == L.P2P_EINVAL
    assert lib.p2p_eval_gravity(*args(L.P2P_GATHER, L.P2P_FP64, -1.0)) == L.P2P_EINVAL
    assert lib.p2p_eval_gravity(*args(L.P2P_GATHER, L.P2P_FP64, float("nan"))) == L.P2P_EINVAL
    assert lib.p2p_eval_gravity(*args(L.P2P_GATHER, L.P2P_FP64, 1e-3)) == L.P2P_OK   # size query
    # single precision throughout is a Helmholtz mode: gravity refuses it
    assert lib.p2p_eval_gravity(*args(L.P2P_GATHER, L.P2P_FP32, 1e-3)) == L.P2P_EUNSUPPORTED
    assert "Helmholtz paths only" in L.last_error()
    # redundant layout without a redundant structure: rejected once the workspace is given
    nb.value = 1 << 20
    st = lib.p2p_eval_gravity(ctypes.byref(t), ctypes.byref(n), None, L.P2P_REDUNDANT, L.P2P_FP64,
                              1e-3, z, z, z, z, z, z, z, z, ctypes.c_void_p(0x100000), ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "needs red" in L.last_error()
    # gravity on a grid tree
    t.kind = L.P2P_TREE_GRIDS
    assert lib.p2p_eval_gravity(*args(L.P2P_GATHER, L.P2P_FP64, 1e-3)) == L.P2P_EINVAL


@pytest.mark.parametrize("prec,eps,ok", [
    (L.P2P_FP32_MIXED, 0.0, True), (L.P2P_FP32_MIXED, 1e-4, True), (L.P2P_FP32_MIXED, 9.9e-5, False),
    (L.P2P_FP32_MIXED, 1e-3, True),
    (L.P2P_FP32_MIXED, 1e-30, False), (L.P2P_FP64, 1e-8, True), (L.P2P_FP64, 1e-3, True),
    (L.P2P_FP64, 1e-30, True), (L.P2P_FP64, 2.0 ** -511, True), (L.P2P_FP64, 1e-160, False),
    (L.P2P_FP64, 5e-324, False)])
def test_eval_rejects_tiny_softening(lib, prec, eps, ok):
    """FP32_MIXED sums the target's own d = 0 term m/eps into a float partial
    and subtracts it again, so a positive eps below 1e-4 would leave more
    rounding in phi than 1e-5 and is refused on the host; FP64 drops that pair
    by position and takes any eps whose square is a normal double (>= 2^-511).
    The same by every gravity entry point that takes eps; eps = 0 stays
    available."""
    t = _tree(10, L_=1)
    t.perm = t.iperm = t.leaf_start = t.leaf_key = t.leaf_level = 0x1000
    n = L.p2p_nbrs()
    n.count, n.nbr_start, n.nbr_idx = 1, 0x1000, 0x1000
    nb = ctypes.c_size_t(0)
    z = ctypes.c_void_p(0x1000)
    want = L.P2P_OK if ok else L.P2P_EINVAL       # OK: the workspace size query went through
    st = lib.p2p_eval_gravity(ctypes.byref(t), ctypes.byref(n), None, L.P2P_GATHER, prec, eps,
                              z, z, z, z, z, z, z, z, None, ctypes.byref(nb), None)
    assert st == want, L.last_error()
    if not ok:
        assert "eps must be 0 or >=" in L.last_error()
    if eps > 0:
        # the FP32_MIXED adjoint needs eps >= 1e-3 (its w^5 terms of close pairs)
        adj_ok = ok and not (prec == L.P2P_FP32_MIXED and eps < 1e-3)
        st = lib.p2p_adjoint(L.P2P_KIND_GRAVITY, ctypes.byref(t), ctypes.byref(n), None, L.P2P_GATHER,
                             prec, eps, None, 0, 1, 0, None, None, None, None, ctypes.byref(nb), None)
        assert st == (L.P2P_OK if adj_ok else L.P2P_EINVAL), L.last_error()


def test_adjoint_unsupported_combinations(lib):
    t = _tree(10, L_=1)
    t.perm = t.iperm = t.leaf_start = t.leaf_key = t.leaf_level = 0x1000
    n = L.p2p_nbrs()
    n.count, n.nbr_start, n.nbr_idx = 1, 0x1000, 0x1000
    nb = ctypes.c_size_t(0)
    st = lib.p2p_adjoint(L.P2P_KIND_GRAVITY, ctypes.byref(t), ctypes.byref(n), None, L.P2P_REDUNDANT,
                         L.P2P_FP64, 1e-3, None, 0, 1, 0, None, None, None, None, ctypes.byref(nb), None)
    assert st == L.P2P_EUNSUPPORTED
    st = lib.p2p_adjoint(L.P2P_KIND_GRAVITY, ctypes.byref(t), ctypes.byref(n), None, L.P2P_GATHER,
                         L.P2P_FP64, 0.0, None, 0, 1, 0, None, None, None, None, ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL
    st = lib.p2p_adjoint(5, ctypes.byref(t), ctypes.byref(n), None, L.P2P_GATHER, L.P2P_FP64, 1e-3,
                         None, 0, 1, 0, None, None, None, None, ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL


def test_interaction_layout_validation(lib):
    t = _tree(10, L_=1)
    t.perm = t.iperm = t.leaf_start = t.leaf_key = t.leaf_level = 0x1000
    n = L.p2p_nbrs()
    n.count, n.nbr_start, n.nbr_idx, n.red_entries = 1, 0x1000, 0x1000, 10
    nb = ctypes.c_size_t(0)
    inter = L.p2p_interactions()
    # size query succeeds on host; a grid tree or a bad precision is rejected
    assert lib.p2p_restructure_interactions(ctypes.byref(t), ctypes.byref(n), None, L.P2P_FP32_MIXED,
                                            ctypes.byref(inter), None, ctypes.byref(nb), None) == L.P2P_OK
    assert nb.value > 0
    assert lib.p2p_restructure_interactions(ctypes.byref(t), ctypes.byref(n), None, 7,
                                            ctypes.byref(inter), None, ctypes.byref(nb), None) == L.P2P_EINVAL
    t.kind = L.P2P_TREE_GRIDS
    st = lib.p2p_restructure_interactions(ctypes.byref(t), ctypes.byref(n), None, L.P2P_FP64,
                                          ctypes.byref(inter), None, ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "particle tree" in L.last_error()
    t.kind = L.P2P_TREE_PARTICLES
    # evaluation: an unbuilt layout, a negative eps, a missing layout
    z = ctypes.c_void_p(0x1000)
    inter.prec = 9
    assert lib.p2p_eval_gravity_interactions(ctypes.byref(t), ctypes.byref(n), ctypes.byref(inter), 1e-3,
                                             z, z, z, z, None, ctypes.byref(nb), None) == L.P2P_EINVAL
    inter.prec = L.P2P_FP64
    assert lib.p2p_eval_gravity_interactions(ctypes.byref(t), ctypes.byref(n), ctypes.byref(inter), -1.0,
                                             z, z, z, z, None, ctypes.byref(nb), None) == L.P2P_EINVAL
    assert lib.p2p_eval_gravity_interactions(ctypes.byref(t), ctypes.byref(n), None, 1e-3,
                                             z, z, z, z, None, ctypes.byref(nb), None) == L.P2P_EINVAL
    assert lib.p2p_eval_gravity_interactions(ctypes.byref(t), ctypes.byref(n), ctypes.byref(inter), 1e-3,
                                             z, z, z, z, None, ctypes.byref(nb), None) == L.P2P_OK


def test_helmholtz_tile_validation(lib):
    n = 16 ** 3
    t = _tree(n, L.P2P_TREE_GRIDS, L_=64)
    t.perm = t.iperm = t.leaf_start = t.leaf_key = t.leaf_level = 0x1000
    t.n_grids, t.key_bits = 1, 4
    g = (L.p2p_grid * 1)()
    g[0].n_side, g[0].h, g[0].k, g[0].point_off = 16, 1 / 16, 1.0, 0
    nl = L.p2p_nbrs()
    nl.count, nl.nbr_start, nl.nbr_idx = 64, 0x1000, 0x1000
    nb = ctypes.c_size_t(0)
    z = ctypes.c_void_p(0x1000)

    def query(tile, nrhs=64, prec=L.P2P_FP32_MIXED):
        tl = (ctypes.c_int32 * 4)(*tile) if tile is not None else None
        return lib.p2p_eval_helmholtz(ctypes.byref(t), ctypes.byref(nl), None, L.P2P_GATHER, prec, g, 1,
                                      nrhs, z, z, tl, None, ctypes.byref(nb), None)
    assert query((4, 2, 64, 1)) == L.P2P_OK
    small = nb.value
    assert query((4, 2, 64, 8)) == L.P2P_OK and nb.value > small    # eight copies of the G blocks
    assert query((4, 2, 64, 3)) == L.P2P_EINVAL and "tile[3]" in L.last_error()
    assert query((3, 2, 64, 1)) == L.P2P_EINVAL and "tile[0]" in L.last_error()
    assert query((4, 0, 64, 1)) == L.P2P_EINVAL and "tile[1]" in L.last_error()
    assert query((4, 2, 64, 1), nrhs=32) == L.P2P_EINVAL and "tile[2]" in L.last_error()
    assert query((4, 2, 32, 1), nrhs=1) == L.P2P_EINVAL          # no tile off the matrix-core path
    assert query(None, nrhs=1) == L.P2P_OK
    assert query((4, 2, 64, 1), prec=L.P2P_FP32) == L.P2P_OK      # single precision throughout
    assert query(None, prec=7) == L.P2P_EINVAL


def test_tile_grain_restructure_validation(lib):
    """The tile grain is refused on particle trees and for grains other than
    2 and 4; a tile-grain layout without its entry rows is refused."""
    t = _tree(1000, L_=10)
    t.perm = t.iperm = t.leaf_start = t.leaf_key = t.leaf_level = 0x1000
    nl = L.p2p_nbrs()
    nl.count, nl.nbr_start, nl.nbr_idx, nl.red_entries = 10, 0x1000, 0x1000, 100
    z = ctypes.c_void_p(0x1000)
    srcs = L.PV4(z, z, z, z)
    nb = ctypes.c_size_t(0)
    red = L.p2p_redundant()
    red.red_start = red.red_self = 0x1000
    red.grain = 2
    st = lib.p2p_restructure_redundant(ctypes.byref(t), ctypes.byref(nl), ctypes.byref(srcs), 1, L.P2P_FP64,
                                       ctypes.byref(red), None, ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "grid trees only" in L.last_error()
    t.kind, t.n_grids, t.key_bits = L.P2P_TREE_GRIDS, 1, 4
    red.grain = 3
    st = lib.p2p_restructure_redundant(ctypes.byref(t), ctypes.byref(nl), ctypes.byref(srcs), 1, L.P2P_FP32,
                                       ctypes.byref(red), None, ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "grain" in L.last_error()
    red.grain = 4
    st = lib.p2p_restructure_redundant(ctypes.byref(t), ctypes.byref(nl), ctypes.byref(srcs), 1, L.P2P_FP32,
                                       ctypes.byref(red), None, ctypes.byref(nb), None)
    assert st == L.P2P_OK and nb.value > 0                        # workspace size
    nb.value = 1 << 20
    st = lib.p2p_restructure_redundant(ctypes.byref(t), ctypes.byref(nl), ctypes.byref(srcs), 1, L.P2P_FP32,
                                       ctypes.byref(red), ctypes.c_void_p(0x100000), ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "red_row" in L.last_error()


def test_periodic_list_validation(lib):
    t = _tree(10, L_=1)
    t.perm = t.iperm = t.leaf_start = t.leaf_key = t.leaf_level = 0x1000
    n = L.p2p_nbrs()
    n.count, n.nbr_start, n.nbr_idx = 1, 0x1000, 0x1000
    nb = ctypes.c_size_t(0)
    z = ctypes.c_void_p(0x1000)

    def grav():
        return lib.p2p_eval_gravity(ctypes.byref(t), ctypes.byref(n), None, L.P2P_GATHER, L.P2P_FP64, 1e-3,
                                    z, z, z, z, z, z, z, z, None, ctypes.byref(nb), None)
    assert grav() == L.P2P_OK
    n.periodic = 1                       # periodic lists need their image codes
    assert grav() == L.P2P_EINVAL and "nbr_shift" in L.last_error()
    n.nbr_shift = 0x1000
    assert grav() == L.P2P_OK
    n.periodic = 2
    assert grav() == L.P2P_EINVAL and "periodic" in L.last_error()
    n.periodic, n.reserved = 1, 1
    assert grav() == L.P2P_EINVAL and "reserved" in L.last_error()
    n.reserved = 0
    # the torus is defined for particle trees only
    t.kind = L.P2P_TREE_GRIDS
    st = lib.p2p_build_neighbors(ctypes.byref(t), ctypes.byref(n), None, ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "particle trees" in L.last_error()
    t.kind = L.P2P_TREE_PARTICLES
    assert lib.p2p_build_neighbors(ctypes.byref(t), ctypes.byref(n), None, ctypes.byref(nb), None) == L.P2P_OK
    plain = nb.value
    n.periodic = 0
    assert lib.p2p_build_neighbors(ctypes.byref(t), ctypes.byref(n), None, ctypes.byref(nb), None) == L.P2P_OK
    assert plain > nb.value             # room for the slot image codes


def test_remote_validation(lib):
    t = _tree(10, L_=1)
    t.perm = t.iperm = t.leaf_start = t.leaf_key = t.leaf_level = 0x1000
    u = _tree(12, L_=2)
    u.perm = u.iperm = u.leaf_start = u.leaf_key = u.leaf_level = 0x2000
    n = L.p2p_nbrs()
    nb = ctypes.c_size_t(0)
    z = ctypes.c_void_p(0x1000)
    # size queries work on the host; a missing or identical source tree is rejected
    assert lib.p2p_build_neighbors_remote(ctypes.byref(t), ctypes.byref(u), ctypes.byref(n), None,
                                          ctypes.byref(nb), None) == L.P2P_OK
    assert lib.p2p_build_neighbors_remote(ctypes.byref(t), None, ctypes.byref(n), None,
                                          ctypes.byref(nb), None) == L.P2P_EINVAL
    assert lib.p2p_build_neighbors_remote(ctypes.byref(t), ctypes.byref(t), ctypes.byref(n), None,
                                          ctypes.byref(nb), None) == L.P2P_EINVAL
    u.kind = L.P2P_TREE_GRIDS
    assert lib.p2p_build_neighbors_remote(ctypes.byref(t), ctypes.byref(u), ctypes.byref(n), None,
                                          ctypes.byref(nb), None) == L.P2P_EINVAL
    assert "particle trees" in L.last_error()
    u.kind = L.P2P_TREE_PARTICLES
    # remote lists may be empty: count 0 is accepted by the evaluation
    n.count, n.nbr_start = 0, 0x1000

    def ev(layout=L.P2P_GATHER, eps=1e-3):
        return lib.p2p_eval_gravity_remote(ctypes.byref(t), ctypes.byref(u), ctypes.byref(n), None, layout,
                                           L.P2P_FP32_MIXED, eps, z, z, z, z, z, z, z, z, z, z, z, None,
                                           ctypes.byref(nb), None)
    assert ev() == L.P2P_OK          # size query (the remote evaluation needs no workspace)
    assert ev(eps=-1.0) == L.P2P_EINVAL
    nb.value = 1 << 20
    st = lib.p2p_eval_gravity_remote(ctypes.byref(t), ctypes.byref(u), ctypes.byref(n), None, L.P2P_REDUNDANT,
                                     L.P2P_FP64, 1e-3, z, z, z, z, z, z, z, z, z, z, z,
                                     ctypes.c_void_p(0x100000), ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "needs red" in L.last_error()


def test_peaks_library_exports_and_rejects_bad_arguments():
    """The microbenchmark library exports every p2pk_ symbol its header
    declares, and refuses bad arguments on the host (no launch, no device)."""
    import ctypes
    src = open(os.path.join(ROOT, "include", "p2p_peaks.h")).read()
    decl = sorted(set(re.findall(r"^\S.*?\b(p2pk_[a-z0-9_]+)\(", src, flags=re.M)))
    assert decl == ["p2pk_mfma_f32", "p2pk_valu_fma", "p2pk_valu_rsq"]
    path = os.path.join(ROOT, "paper_2511_21535_amd", "libp2p_peaks.so")
    if not os.path.exists(path):
        from paper_2511_21535_amd import build
        build.build()
    pk = ctypes.CDLL(path)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: the checks come first
    for name in decl:
        fn = getattr(pk, name)
        fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]
        fn.restype = ctypes.c_int
        assert fn(None, 8, 1, None) == -1
        assert fn(fake, 0, 1, None) == -1
        assert fn(fake, 8, 0, None) == -1


def test_helmholtz_plan_host_checks(lib):
    """p2p_helmholtz_prepare with plan->buf == NULL only sizes the plan (the
    G blocks of every distinct k h, float4 entries with several RHS); an
    unprepared plan, or one whose fingerprint is of other arguments, is refused
    on the host by p2p_eval_helmholtz_prepared."""
    n = 16 ** 3
    t = _tree(n, L.P2P_TREE_GRIDS, L_=64)
    t.perm = t.iperm = t.leaf_start = t.leaf_key = t.leaf_level = 0x1000
    t.n_grids, t.key_bits = 1, 4
    g = (L.p2p_grid * 1)()
    g[0].n_side, g[0].h, g[0].k, g[0].point_off = 16, 1 / 16, 1.0, 0
    nl = L.p2p_nbrs()
    nl.count, nl.nbr_start, nl.nbr_idx = 64, 0x1000, 0x1000
    z = ctypes.c_void_p(0x1000)
    p = L.p2p_helmholtz_plan()
    assert lib.p2p_helmholtz_prepare(ctypes.byref(t), ctypes.byref(nl), L.P2P_FP32_MIXED, g, 1, 1, None,
                                     ctypes.byref(p), None) == L.P2P_OK
    one = p.bytes
    assert one >= 27 * 64 * 64 * 8 and p.fingerprint == 0     # one set of G blocks; nothing prepared
    assert lib.p2p_helmholtz_prepare(ctypes.byref(t), ctypes.byref(nl), L.P2P_FP32_MIXED, g, 1, 64, None,
                                     ctypes.byref(p), None) == L.P2P_OK
    assert p.bytes > one                       # float4 G entries (sums of the three-product form)
    nb = ctypes.c_size_t(0)
    st = lib.p2p_eval_helmholtz_prepared(ctypes.byref(t), ctypes.byref(nl), None, L.P2P_GATHER, g, 1,
                                         ctypes.byref(p), z, z, None, ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "not prepared" in L.last_error()
    p.buf, p.fingerprint, p.prec, p.nrhs = 0x1000, 12345, L.P2P_FP32_MIXED, 1
    st = lib.p2p_eval_helmholtz_prepared(ctypes.byref(t), ctypes.byref(nl), None, L.P2P_GATHER, g, 1,
                                         ctypes.byref(p), z, z, None, ctypes.byref(nb), None)
    assert st == L.P2P_EINVAL and "prepared for another" in L.last_error()

"""FP64 CPU oracle for the MLFMA near-field (P2P) operator -- ctypes wrapper.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU library
and its Python binding never import it; the two share no code.

The C source (``p2p_oracle.c``) is the plain definition of each step; this
module only marshals numpy arrays.  Every function names the paper passage it
follows (arXiv 2511.21535), or the reading taken where the paper is silent.

Pins: the tests in ``tests/test_oracle_*.py`` check every function here against
closed forms, invariants, hand-computed values and brute force, not against
itself.  Parity unpinned: the Locality metric's absolute values (the paper's
dispersion formulas in Table 5 are garbled); only its D = 1 and V' = N/S
special cases are pinned.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "p2p_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


_FLAGS = ["-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, -O3; no -march=native, so the
    library built here runs on any x86-64 host)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def use_native(directory: str) -> str:
    """Compile the same source with -O3 -march=native for the host it runs on,
    into `directory`, and load that build in place of the portable one (for
    timing the oracle on the host's cores; the arithmetic is the same C code).
    Returns the gcc command line."""
    global _lib
    out = os.path.join(directory, "liboracle_native.so")
    cmd = ["gcc", *_FLAGS, "-march=native", _SRC, "-o", out, "-lm"]
    subprocess.check_call(cmd)
    lib = ctypes.CDLL(out)
    _declare(lib)
    _lib = lib
    return " ".join(cmd[:-4] + ["p2p_oracle.c"])


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
F64 = ctypes.c_double


def _declare(lib):
    lib.orc_threads.restype = ctypes.c_int
    lib.orc_threads.argtypes = []
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_morton3.restype = ctypes.c_uint64
    lib.orc_morton3.argtypes = [ctypes.c_uint32] * 3 + [ctypes.c_int]
    lib.orc_particle_keys.restype = I64
    lib.orc_particle_keys.argtypes = [I64, P, P, P, P]
    lib.orc_grid_bits.restype = I32
    lib.orc_grid_bits.argtypes = [I32, P]
    lib.orc_grid_keys.restype = None
    lib.orc_grid_keys.argtypes = [I32, P, P, P]
    lib.orc_build_tree_particles.restype = I64
    lib.orc_build_tree_particles.argtypes = [I64, P, I32, I32, P, P, P, P, P, P]
    lib.orc_build_tree_grids.restype = I64
    lib.orc_build_tree_grids.argtypes = [I32, P, P, I64, P, P, P, P, P, P, P, P]
    lib.orc_neighbors.restype = I64
    lib.orc_neighbors.argtypes = [I64, P, P, P, P, I64, P, P, I64]
    lib.orc_red_offsets.restype = I64
    lib.orc_red_offsets.argtypes = [I64, P, P, P, P, P, P]
    lib.orc_restructure_rows.restype = None
    lib.orc_restructure_rows.argtypes = [I64, P, P, P, P, P, P, I64, P]
    lib.orc_restructure_gravity_rel.restype = None
    lib.orc_restructure_gravity_rel.argtypes = [I64, P, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_restructure_gravity_rows.restype = None
    lib.orc_restructure_gravity_rows.argtypes = [I64, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_restructure_interactions.restype = I64
    lib.orc_restructure_interactions.argtypes = [I64, P, P, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_neighbors_cross.restype = I64
    lib.orc_neighbors_cross.argtypes = [I64, P, P, I64, P, P, I32, P, P, P, I64]
    lib.orc_gravity_remote.restype = None
    lib.orc_gravity_remote.argtypes = [I64, P, P, P, P, P, P, P, P, P, P, P, F64, P, P, P, P, P, P, P]
    lib.orc_neighbors_periodic.restype = I64
    lib.orc_neighbors_periodic.argtypes = [I64, P, P, P, I64, P, P, P, I64]
    lib.orc_gravity_leaves.restype = I64
    lib.orc_gravity_leaves.argtypes = [P, P, P, P, F64, P, P, P, I64, P, P, P, P, P, P, P, P]
    lib.orc_gravity_adjoint_leaves.restype = I64
    lib.orc_gravity_adjoint_leaves.argtypes = ([P] * 4 + [F64] + [P] * 4 + [P, P, P, I64, P, P, P]
                                               + [P] * 5)
    lib.orc_helmholtz.restype = None
    lib.orc_helmholtz.argtypes = [I32, P, P, P, P, I32, P, P, I64, P]
    lib.orc_helmholtz_transpose.restype = None
    lib.orc_helmholtz_transpose.argtypes = [I32, P, P, P, P, I64, I32, P, P]
    lib.orc_tile_layout.restype = I64
    lib.orc_tile_layout.argtypes = [I64, P, P, P, I32, P, P, P, P, P, P, P, I64, P]
    lib.orc_locality.restype = None
    lib.orc_locality.argtypes = [I64, P, P, I64, I64, F64, F64, P]


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(_load().orc_threads())


def set_threads(n: int) -> None:
    """Sets the OpenMP threads of the oracle's parallel loops."""
    _load().orc_set_threads(int(n))


# ---------------------------------------------------------------------------
# Keys and trees
# ---------------------------------------------------------------------------
def morton3(x: int, y: int, z: int, bits: int) -> int:
    """Bit interleave, x least significant (the ordering this
    library reads into the paper, which fixes none: leaves in ascending key order)."""
    return int(_load().orc_morton3(x, y, z, bits))


def particle_keys(x, y, z):
    """Depth-20 Morton keys of particles in [0,1)^3.  Returns (keys, n_bad)."""
    x, y, z = (_c(v, np.float64) for v in (x, y, z))
    key = np.zeros(x.shape[0], dtype=np.uint64)
    bad = _load().orc_particle_keys(x.shape[0], _p(x), _p(y), _p(z), _p(key))
    return key, int(bad)


def grid_bits(n_side) -> int:
    n_side = _c(n_side, np.int32)
    return int(_load().orc_grid_bits(n_side.shape[0], _p(n_side)))


def grid_offsets(n_side):
    n_side = np.asarray(n_side, dtype=np.int64)
    off = np.zeros(n_side.shape[0] + 1, dtype=np.int64)
    off[1:] = np.cumsum(n_side ** 3)
    return off


def grid_keys(n_side):
    n_side = _c(n_side, np.int32)
    off = grid_offsets(n_side)
    key = np.zeros(int(off[-1]), dtype=np.uint64)
    _load().orc_grid_keys(n_side.shape[0], _p(n_side), _p(off), _p(key))
    return key


class Tree:
    """Oracle tree: perm, leaf_start, leaf_key, leaf_level (the boundary's
    outputs) plus anchor/size/inst, which only the oracle keeps."""

    def __init__(self, perm, leaf_start, leaf_key, leaf_level, anchor, size, inst, kind):
        self.perm, self.leaf_start, self.leaf_key, self.leaf_level = perm, leaf_start, leaf_key, leaf_level
        self.anchor, self.size, self.inst, self.kind = anchor, size, inst, kind

    @property
    def n_leaves(self):
        return self.leaf_key.shape[0]

    @property
    def occ(self):
        return np.diff(self.leaf_start)


def build_tree_particles(x, y, z, depth: int, leaf_cap: int) -> Tree:
    """Octree over the unit cube (Sec. 5.2: an irregular tree rebuilt every
    step; the split rule the paper leaves open is read as: split iff
    count > leaf_cap and level < depth; leaf_cap = 0
    means a uniform tree of depth `depth`)."""
    key, bad = particle_keys(x, y, z)
    if bad:
        raise ValueError(f"{bad} points outside [0,1)^3")
    n = key.shape[0]
    perm = np.zeros(n, dtype=np.int32)
    ls = np.zeros(n + 1, dtype=np.int32)
    lk = np.zeros(max(n, 1), dtype=np.uint64)
    ll = np.zeros(max(n, 1), dtype=np.int8)
    an = np.zeros((max(n, 1), 3), dtype=np.int32)
    sz = np.zeros(max(n, 1), dtype=np.int32)
    L = _load().orc_build_tree_particles(n, _p(key), depth, leaf_cap, _p(perm), _p(ls), _p(lk),
                                         _p(ll), _p(an), _p(sz))
    return Tree(perm, ls[: L + 1].copy(), lk[:L].copy(), ll[:L].copy(), an[:L].copy(),
                sz[:L].copy(), None, "particles")


def build_tree_grids(n_side) -> Tree:
    """Boxes of 4x4x4 grid points (Sec. 5.1: a regular tree over a uniform
    mesh), boxes and points in Morton order."""
    n_side = _c(n_side, np.int32)
    off = grid_offsets(n_side)
    key = grid_keys(n_side)
    n = key.shape[0]
    perm = np.zeros(n, dtype=np.int32)
    ls = np.zeros(n + 1, dtype=np.int32)
    Lmax = n // 64 + 1
    lk = np.zeros(Lmax, dtype=np.uint64)
    ll = np.zeros(Lmax, dtype=np.int8)
    an = np.zeros((Lmax, 3), dtype=np.int32)
    sz = np.zeros(Lmax, dtype=np.int32)
    inst = np.zeros(Lmax, dtype=np.int32)
    L = _load().orc_build_tree_grids(n_side.shape[0], _p(n_side), _p(off), n, _p(key), _p(perm),
                                     _p(ls), _p(lk), _p(ll), _p(an), _p(sz), _p(inst))
    return Tree(perm, ls[: L + 1].copy(), lk[:L].copy(), ll[:L].copy(), an[:L].copy(),
                sz[:L].copy(), inst[:L].copy(), "grids")


def neighbors(tree: Tree, targets=None):
    """Near lists (the E2 neighbourhood, Sec. 5.1, read for adaptive trees as: leaves whose
    closed cubes touch, the leaf itself included, ascending).  Brute force
    over all leaves.  Returns (nbr_start int64 [T+1], nbr_idx int32 [E])."""
    L = tree.n_leaves
    if targets is None:
        targets = np.arange(L, dtype=np.int32)
    targets = _c(targets, np.int32)
    T = targets.shape[0]
    start = np.zeros(T + 1, dtype=np.int64)
    lib = _load()
    inst = tree.inst if tree.inst is not None else None
    total = lib.orc_neighbors(L, _p(tree.anchor), _p(tree.size), _p(inst), _p(targets), T,
                              _p(start), None, 0)
    idx = np.zeros(max(total, 1), dtype=np.int32)
    lib.orc_neighbors(L, _p(tree.anchor), _p(tree.size), _p(inst), _p(targets), T, _p(start),
                      _p(idx), total)
    return start, idx[:total]


def neighbors_periodic(tree: Tree, targets=None):
    """Periodic near lists on the unit torus (the periodic interactions of
    Sec. 5.2, read as): every (leaf B,
    image c) whose cube shifted by image c touches A's, ascending in (c, B);
    image code c = (sx+1) + 3 (sy+1) + 9 (sz+1) shifts a source by
    (sx, sy, sz) domain edges, 13 = unshifted.  Brute force.  Returns
    (nbr_start int64 [T+1], nbr_idx int32 [E], nbr_shift int8 [E])."""
    if tree.kind != "particles":
        raise ValueError("periodic images are defined for particle trees only")
    L = tree.n_leaves
    if targets is None:
        targets = np.arange(L, dtype=np.int32)
    targets = _c(targets, np.int32)
    T = targets.shape[0]
    start = np.zeros(T + 1, dtype=np.int64)
    lib = _load()
    total = lib.orc_neighbors_periodic(L, _p(tree.anchor), _p(tree.size), _p(targets), T,
                                       _p(start), None, None, 0)
    idx = np.zeros(max(total, 1), dtype=np.int32)
    sh = np.zeros(max(total, 1), dtype=np.int8)
    lib.orc_neighbors_periodic(L, _p(tree.anchor), _p(tree.size), _p(targets), T, _p(start),
                               _p(idx), _p(sh), total)
    return start, idx[:total], sh[:total]


def neighbors_remote(tree: Tree, src_tree: Tree, periodic: bool = False, targets=None):
    """Remote near lists (Sec. 5.2, remote interactions): for every leaf of
    `tree` (or the leaves `targets`, in that order), the leaves of `src_tree`
    (another particle set) whose cubes touch it, through the periodic images
    when `periodic`, ascending in (code, B).  Returns (nbr_start, nbr_idx,
    nbr_shift)."""
    if tree.kind != "particles" or src_tree.kind != "particles":
        raise ValueError("remote lists are defined for particle trees")
    anchor, size = tree.anchor, tree.size
    if targets is not None:
        sel = np.asarray(targets, dtype=np.int64)
        anchor, size = _c(anchor[sel], np.int32), _c(size[sel], np.int32)
    Lt, Ls = anchor.shape[0], src_tree.n_leaves
    start = np.zeros(Lt + 1, dtype=np.int64)
    lib = _load()
    args = (Lt, _p(anchor), _p(size), Ls, _p(src_tree.anchor), _p(src_tree.size), int(periodic))
    total = lib.orc_neighbors_cross(*args, _p(start), None, None, 0)
    idx = np.zeros(max(total, 1), dtype=np.int32)
    sh = np.zeros(max(total, 1), dtype=np.int8)
    lib.orc_neighbors_cross(*args, _p(start), _p(idx), _p(sh), total)
    return start, idx[:total], sh[:total]


def restructure_remote(tree: Tree, src_tree: Tree, nbr, sx, sy, sz, sm, prec="fp64"):
    """Redundant layout of remote sources: (red_start, rows) with the segment
    of target leaf A holding, for the entries of its remote list in order, the
    source points of leaf B of `src_tree` at their image: float64 [S, 4]
    (x + s, y + s, z + s, m), or for "fp32" float32 relative to the centre of
    A as in restructure_gravity_rel."""
    start, idx, sh = nbr
    occ = np.diff(src_tree.leaf_start).astype(np.int64)
    seg = np.array([occ[idx[start[a]:start[a + 1]]].sum() for a in range(tree.n_leaves)], dtype=np.int64)
    rs = np.concatenate([[0], np.cumsum(seg)]).astype(np.int64)
    S = int(rs[-1])
    arrs = [_c(v, np.float64) for v in (sx, sy, sz, sm)]
    args = (tree.n_leaves, _p(src_tree.leaf_start), _p(src_tree.perm), _p(_c(start, np.int64)),
            _p(_c(idx, np.int32)), _shift_arg(sh), _p(rs))
    if prec == "fp64":
        out = np.zeros((max(S, 1), 4), dtype=np.float64)
        _load().orc_restructure_gravity_rows(*args, *[_p(a) for a in arrs], _p(out))
    else:
        out = np.zeros((max(S, 1), 4), dtype=np.float32)
        _load().orc_restructure_gravity_rel(*args, _p(tree.anchor), _p(tree.size), *[_p(a) for a in arrs],
                                            _p(out))
    return rs, out[:S]


def gravity_remote(x, y, z, tree: Tree, sx, sy, sz, sm, src_tree: Tree, eps, nbr):
    """Remote gravity: for every point of the target set (caller order), the
    sums over the source points of the leaves in its leaf's remote list, each
    at its image; no pair is skipped.  Returns (phi, ax, ay, az)."""
    x, y, z = (_c(v, np.float64) for v in (x, y, z))
    sx, sy, sz, sm = (_c(v, np.float64) for v in (sx, sy, sz, sm))
    start, idx, sh = nbr
    outs = [np.zeros(len(x)) for _ in range(4)]
    _load().orc_gravity_remote(tree.n_leaves, _p(tree.perm), _p(tree.leaf_start), _p(x), _p(y), _p(z),
                               _p(src_tree.perm), _p(src_tree.leaf_start), _p(sx), _p(sy), _p(sz), _p(sm),
                               float(eps), _p(_c(start, np.int64)), _p(_c(idx, np.int32)),
                               _shift_arg(sh), *[_p(o) for o in outs])
    return tuple(outs)


def shift_vectors(codes):
    """Image codes -> shift vectors (sx, sy, sz) in domain edges, float64 [E, 3]."""
    c = np.asarray(codes, dtype=np.int64)
    return np.stack([c % 3 - 1, (c // 3) % 3 - 1, c // 9 - 1], axis=-1).astype(np.float64)


def _shift_arg(nbr_shift):
    return None if nbr_shift is None else _p(_c(nbr_shift, np.int8))


# ---------------------------------------------------------------------------
# Redundant layout
# ---------------------------------------------------------------------------
def red_offsets(tree: Tree, nbr_start, nbr_idx, nbr_shift=None):
    """Segment starts and self offsets of the redundant layout (Sec. 5.2.1:
    data duplicated so each target reads one contiguous block).  With image
    codes the self offset is that of the unshifted image of A."""
    L = tree.n_leaves
    rs = np.zeros(L + 1, dtype=np.int64)
    self_ = np.zeros(max(L, 1), dtype=np.int32)
    S = _load().orc_red_offsets(L, _p(tree.leaf_start), _p(_c(nbr_start, np.int64)),
                                _p(_c(nbr_idx, np.int32)), _shift_arg(nbr_shift), _p(rs),
                                _p(self_))
    return rs, self_[:L].copy(), int(S)


def restructure_rows(tree: Tree, nbr_start, nbr_idx, red_start, src):
    """Copy rows of `src` (caller order, first axis = point) into the
    redundant layout, bit for bit."""
    src = np.ascontiguousarray(src)
    row_bytes = src.strides[0] if src.ndim > 0 else src.itemsize
    S = int(red_start[-1])
    out = np.zeros((S,) + src.shape[1:], dtype=src.dtype)
    _load().orc_restructure_rows(tree.n_leaves, _p(tree.leaf_start), _p(tree.perm),
                                 _p(_c(nbr_start, np.int64)), _p(_c(nbr_idx, np.int32)),
                                 _p(_c(red_start, np.int64)), _p(src), row_bytes, _p(out))
    return out


def tile_layout(tree: Tree, nbr_start, nbr_idx, grain: int):
    """Block-level redundancy on a grid tree (Sec. 3.5: for dense, regular
    distributions, data duplicated per thread block rather than per thread):
    tiles of grain^3 boxes, each with one segment holding the rows of the union
    of its boxes' near lists.  Returns (tile_first int32 [T+1], halo_start
    int64 [T+1], halo_idx int32 [H], seg_start int64 [T+1], red_row int64 [E]):
    the tiles' first boxes, the halo boxes of each tile (ascending), the first
    row of each tile's segment, and for every near-list entry (A, B) the first
    row of B in the segment of A's tile."""
    if tree.kind != "grids":
        raise ValueError("tiles are defined on grid trees")
    L = tree.n_leaves
    nbr_start, nbr_idx = _c(nbr_start, np.int64), _c(nbr_idx, np.int32)
    tf = np.zeros(L + 1, dtype=np.int32)
    hs = np.zeros(L + 1, dtype=np.int64)
    ss = np.zeros(L + 1, dtype=np.int64)
    H = ctypes.c_int64(0)
    lib = _load()
    args = (L, _p(tree.anchor), _p(tree.inst), _p(tree.leaf_start), int(grain), _p(nbr_start), _p(nbr_idx),
            _p(tf), _p(hs), _p(ss))
    lib.orc_tile_layout(*args, None, None, 0, ctypes.byref(H))
    hi = np.zeros(max(H.value, 1), dtype=np.int32)
    rr = np.zeros(max(nbr_idx.shape[0], 1), dtype=np.int64)
    T = lib.orc_tile_layout(*args, _p(hi), _p(rr), H.value, ctypes.byref(H))
    return tf[:T + 1].copy(), hs[:T + 1].copy(), hi[:H.value].copy(), ss[:T + 1].copy(), rr[:nbr_idx.shape[0]].copy()


def restructure_tile_rows(tree: Tree, halo_start, halo_idx, seg_start, src):
    """The payload of the tile segments: for each tile, the rows of `src`
    (caller order) of its halo boxes' sorted slots, bit for bit."""
    src = np.ascontiguousarray(src)
    row_bytes = src.strides[0] if src.ndim > 0 else src.itemsize
    out = np.zeros((int(seg_start[-1]),) + src.shape[1:], dtype=src.dtype)
    _load().orc_restructure_rows(len(halo_start) - 1, _p(tree.leaf_start), _p(tree.perm),
                                 _p(_c(halo_start, np.int64)), _p(_c(halo_idx, np.int32)),
                                 _p(_c(seg_start, np.int64)), _p(src), row_bytes, _p(out))
    return out


def restructure_gravity_rel(tree: Tree, nbr_start, nbr_idx, red_start, x, y, z, m,
                            nbr_shift=None):
    """FP32-mixed redundant payload: float32 [S, 4] rows (x + s - c_A, y + s -
    c_A, z + s - c_A, m) with c_A the centre of the segment's target leaf and
    s the entry's image shift, the position taken in double and rounded to
    single once."""
    S = int(red_start[-1])
    out = np.zeros((max(S, 1), 4), dtype=np.float32)
    arrs = [_c(v, np.float64) for v in (x, y, z, m)]
    _load().orc_restructure_gravity_rel(tree.n_leaves, _p(tree.leaf_start), _p(tree.perm),
                                        _p(_c(nbr_start, np.int64)), _p(_c(nbr_idx, np.int32)),
                                        _shift_arg(nbr_shift), _p(_c(red_start, np.int64)),
                                        _p(tree.anchor), _p(tree.size),
                                        *[_p(a) for a in arrs], _p(out))
    return out[:S]


def restructure_gravity_rows(tree: Tree, nbr_start, nbr_idx, red_start, x, y, z, m,
                             nbr_shift=None):
    """FP64 redundant payload: float64 [S, 4] rows (x + s, y + s, z + s, m)
    with s the entry's image shift (zero without image codes)."""
    S = int(red_start[-1])
    out = np.zeros((max(S, 1), 4), dtype=np.float64)
    arrs = [_c(v, np.float64) for v in (x, y, z, m)]
    _load().orc_restructure_gravity_rows(tree.n_leaves, _p(tree.leaf_start), _p(tree.perm),
                                         _p(_c(nbr_start, np.int64)), _p(_c(nbr_idx, np.int32)),
                                         _shift_arg(nbr_shift), _p(_c(red_start, np.int64)),
                                         *[_p(a) for a in arrs], _p(out))
    return out[:S]


def restructure_interactions(tree: Tree, nbr_start, nbr_idx, x, y, z, m, prec="fp64",
                             nbr_shift=None):
    """Per-interaction layout (Sec. 5.2.1): (rec_start [E+1], rows) with one
    record per near-list entry (A, B): header (occ_A, occ_B, A, B), A's rows,
    B's rows.  prec "fp64": float64 [rows, 4], header as doubles; "fp32":
    float32 [rows, 4] relative to the centre of A, header as int32 bits."""
    ns, ni = _c(nbr_start, np.int64), _c(nbr_idx, np.int32)
    E = int(ns[-1])
    rec = np.zeros(E + 1, dtype=np.int64)
    arrs = [_c(v, np.float64) for v in (x, y, z, m)]
    lib = _load()
    args = (tree.n_leaves, _p(tree.leaf_start), _p(tree.perm), _p(ns), _p(ni),
            _shift_arg(nbr_shift), _p(tree.anchor), _p(tree.size), *[_p(a) for a in arrs], _p(rec))
    rows = lib.orc_restructure_interactions(*args, None, None)
    if prec == "fp64":
        out = np.zeros((max(rows, 1), 4), dtype=np.float64)
        lib.orc_restructure_interactions(*args, _p(out), None)
    else:
        out = np.zeros((max(rows, 1), 4), dtype=np.float32)
        lib.orc_restructure_interactions(*args, None, _p(out))
    return rec, out[:rows]


# ---------------------------------------------------------------------------
# Gravity
# ---------------------------------------------------------------------------
def gravity_leaves(x, y, z, m, eps, tree: Tree, sel, sel_nbr_start, sel_nbr_idx,
                   sel_nbr_shift=None):
    """Near-field gravity for the particles of the selected leaves (the paper
    gives no gravity law; read as G = 1, phi negative, Plummer softening; with image codes each source sits
    at x_j + s).  Returns (caller idx, phi, ax, ay, az)."""
    x, y, z, m = (_c(v, np.float64) for v in (x, y, z, m))
    sel = _c(sel, np.int32)
    occ = np.diff(tree.leaf_start)
    T = int(occ[sel].sum()) if sel.shape[0] else 0
    idx = np.zeros(max(T, 1), dtype=np.int32)
    outs = [np.zeros(max(T, 1)) for _ in range(4)]
    _load().orc_gravity_leaves(_p(x), _p(y), _p(z), _p(m), float(eps), _p(tree.perm),
                               _p(tree.leaf_start), _p(sel), sel.shape[0],
                               _p(_c(sel_nbr_start, np.int64)), _p(_c(sel_nbr_idx, np.int32)),
                               _shift_arg(sel_nbr_shift), _p(idx), *[_p(o) for o in outs])
    return (idx[:T],) + tuple(o[:T] for o in outs)


def gravity(x, y, z, m, eps, tree: Tree, nbr=None):
    """Near-field gravity for every particle, in caller order.  `nbr` is
    (nbr_start, nbr_idx) or, with periodic images, (.., .., nbr_shift)."""
    if nbr is None:
        nbr = neighbors(tree)
    sel = np.arange(tree.n_leaves, dtype=np.int32)
    idx, p, ax, ay, az = gravity_leaves(x, y, z, m, eps, tree, sel, *nbr)
    n = len(x)
    out = [np.zeros(n) for _ in range(4)]
    for o, v in zip(out, (p, ax, ay, az)):
        o[idx] = v
    return tuple(out)


def gravity_adjoint_leaves(x, y, z, m, eps, gp, gax, gay, gaz, tree: Tree, sel, sel_nbr_start,
                           sel_nbr_idx, sel_nbr_shift=None):
    """Reverse-mode derivative of near-field gravity w.r.t. m and x for the
    particles of the selected leaves.  Returns (caller idx, gm, gx, gy, gz)."""
    arrs = [_c(v, np.float64) for v in (x, y, z, m, gp, gax, gay, gaz)]
    sel = _c(sel, np.int32)
    occ = np.diff(tree.leaf_start)
    T = int(occ[sel].sum()) if sel.shape[0] else 0
    idx = np.zeros(max(T, 1), dtype=np.int32)
    outs = [np.zeros(max(T, 1)) for _ in range(4)]
    _load().orc_gravity_adjoint_leaves(*[_p(a) for a in arrs[:4]], float(eps),
                                       *[_p(a) for a in arrs[4:]], _p(tree.perm),
                                       _p(tree.leaf_start), _p(sel), sel.shape[0],
                                       _p(_c(sel_nbr_start, np.int64)),
                                       _p(_c(sel_nbr_idx, np.int32)),
                                       _shift_arg(sel_nbr_shift), _p(idx),
                                       *[_p(o) for o in outs])
    return (idx[:T],) + tuple(o[:T] for o in outs)


def gravity_adjoint(x, y, z, m, eps, gp, gax, gay, gaz, tree: Tree, nbr=None):
    if nbr is None:
        nbr = neighbors(tree)
    sel = np.arange(tree.n_leaves, dtype=np.int32)
    idx, gm, gx, gy, gz = gravity_adjoint_leaves(x, y, z, m, eps, gp, gax, gay, gaz, tree, sel,
                                                 *nbr)
    n = len(x)
    out = [np.zeros(n) for _ in range(4)]
    for o, v in zip(out, (gm, gx, gy, gz)):
        o[idx] = v
    return tuple(out)


# ---------------------------------------------------------------------------
# Helmholtz
# ---------------------------------------------------------------------------
def _grid_args(n_side, h=None, kw=None):
    n_side = _c(n_side, np.int32)
    if h is None:
        h = 1.0 / n_side.astype(np.float64)
    if kw is None:
        kw = 2.0 * np.pi / (10.0 * np.asarray(h, dtype=np.float64))
    off = grid_offsets(n_side)
    return n_side, _c(h, np.float64), _c(kw, np.float64), off


def helmholtz(n_side, q, targets=None, h=None, kw=None):
    """u_I = sum_{J near I, J != I} e^{ik r}/(4 pi r) q_J on regular grids
    (Sec. 5.1, read as the 3-D kernel on cell-centred points, k = 2 pi/(10 h)).
    q: complex [N, nrhs] (or [N]) in caller order.  Returns complex128
    [len(targets), nrhs] (or [len(targets)])."""
    n_side, h, kw, off = _grid_args(n_side, h, kw)
    q = np.asarray(q)
    vec = q.ndim == 1
    q2 = _c(q.reshape(q.shape[0], -1), np.complex128)
    n, nrhs = q2.shape
    if targets is None:
        targets = np.arange(n, dtype=np.int64)
    targets = _c(targets, np.int64)
    u = np.zeros((targets.shape[0], nrhs), dtype=np.complex128)
    _load().orc_helmholtz(n_side.shape[0], _p(n_side), _p(h), _p(kw), _p(off), nrhs, _p(q2),
                          _p(targets), targets.shape[0], _p(u))
    return u[:, 0] if vec else u


def helmholtz_transpose(n_side, g, h=None, kw=None):
    """(A^T g)_J = sum_I A_IJ g_I by scattering (adjoint of the near-field
    Helmholtz operator)."""
    n_side, h, kw, off = _grid_args(n_side, h, kw)
    g = np.asarray(g)
    vec = g.ndim == 1
    g2 = _c(g.reshape(g.shape[0], -1), np.complex128)
    n, nrhs = g2.shape
    out = np.zeros((n, nrhs), dtype=np.complex128)
    _load().orc_helmholtz_transpose(n_side.shape[0], _p(n_side), _p(h), _p(kw), _p(off), n, nrhs,
                                    _p(g2), _p(out))
    return out[:, 0] if vec else out


# ---------------------------------------------------------------------------
# Locality
# ---------------------------------------------------------------------------
def locality(nbr_start, nbr_idx, n, S, bytes_per_entry, cache_bytes):
    """Definition 1 with Formulas (10)/(11) (Sec. 3.4), read as: D = runs
    of consecutive leaf ids, V = whole footprint per layout, C = cache bytes."""
    out = np.zeros(6)
    nbr_start = _c(nbr_start, np.int64)
    _load().orc_locality(nbr_start.shape[0] - 1, _p(nbr_start), _p(_c(nbr_idx, np.int32)), n, S,
                         float(bytes_per_entry), float(cache_bytes), _p(out))
    keys = ["D_mean", "V_gather", "V_red", "D_ratio", "V_ratio", "locality"]
    return dict(zip(keys, out.tolist()))


def pair_count(tree: Tree, nbr_start, nbr_idx):
    """Ordered near pairs, self excluded: sum_A occ(A) sum_{B in nbr(A)} occ(B) - N."""
    occ = np.diff(tree.leaf_start).astype(np.int64)
    seg = np.add.reduceat(occ[nbr_idx], nbr_start[:-1]) if nbr_idx.shape[0] else np.zeros(0)
    seg = np.where(np.diff(nbr_start) > 0, seg, 0)
    return int((occ * seg).sum() - occ.sum())

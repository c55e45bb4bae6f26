"""Torch-facing API of libp2p: device memory from torch, work on torch's
current stream, every step in the library's HIP kernels.

    tree = Tree.build_particles(x, y, z, depth=20, leaf_cap=64)
    nbrs = tree.neighbors()
    red  = restructure_gravity(tree, nbrs, x, y, z, m, prec="fp32")
    phi, ax, ay, az = gravity(tree, nbrs, eps, x=x, y=y, z=z, m=m)                 # gather
    phi, ax, ay, az = gravity(tree, nbrs, eps, red=red, layout="redundant", prec="fp32")

Nothing here computes any part of the operator on the host or with torch
arithmetic; torch only allocates and provides the stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib as L

# "fp32" and "fp32_mixed": single-precision pair terms, double-precision
# per-target sums; "fp32_plain" (Helmholtz): single precision throughout
PREC = {"fp64": L.P2P_FP64, "fp32": L.P2P_FP32_MIXED, "fp32_mixed": L.P2P_FP32_MIXED, "fp32_plain": L.P2P_FP32}
LAYOUT = {"gather": L.P2P_GATHER, "redundant": L.P2P_REDUNDANT}


def _require_device(t: torch.Tensor, name: str, dtype=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t


def _vec(t: Optional[torch.Tensor], name: str, n: int, dtype=torch.float64, optional: bool = False):
    """A per-point array the kernels index up to n: a contiguous GPU tensor of
    that dtype with exactly n elements (n x nrhs for right-hand sides); a host
    pointer or a short array would reach the kernels unchecked."""
    if t is None:
        if optional:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    return t


def _outs(out, n: int, dev):
    """The four float64 result arrays: allocated, or the caller's, checked."""
    if out is None:
        return [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4)]
    if len(out) != 4:
        raise ValueError("out must hold four arrays (phi, ax, ay, az)")
    for nm, o in zip(("phi", "ax", "ay", "az"), out):
        _vec(o, nm, n)
    return out


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(call, device) -> Tuple[torch.Tensor, ctypes.c_size_t]:
    """Run `call(ws, ws_bytes)` once with ws = NULL to size the workspace,
    allocate it from torch, and return it with its size."""
    nbytes = ctypes.c_size_t(0)
    L.check(call(None, ctypes.byref(nbytes)))
    ws = torch.empty(max(int(nbytes.value), 256), dtype=torch.uint8, device=device)
    nbytes = ctypes.c_size_t(ws.numel())
    return ws, nbytes


def _call(call, device):
    ws, nbytes = _workspace(call, device)
    st = call(_ptr(ws), ctypes.byref(nbytes))
    return st, ws


@dataclass
class Grid:
    """One grid instance: n_side^3 cell-centred points, spacing h, wavenumber k."""
    n_side: int
    h: float
    k: float


def grids_struct(grids: Sequence[Grid]):
    arr = (L.p2p_grid * len(grids))()
    off = 0
    for i, g in enumerate(grids):
        arr[i].n_side = int(g.n_side)
        arr[i].reserved = 0
        arr[i].h = float(g.h)
        arr[i].k = float(g.k)
        arr[i].point_off = off
        off += int(g.n_side) ** 3
    return arr, off


@dataclass
class Tree:
    n: int
    n_leaves: int
    kind: int
    key_bits: int
    max_level: int
    perm: torch.Tensor
    leaf_start: torch.Tensor
    leaf_key: torch.Tensor
    leaf_level: torch.Tensor
    iperm: torch.Tensor
    grids: List[Grid] = field(default_factory=list)

    def struct(self) -> L.p2p_tree:
        t = L.p2p_tree()
        t.n, t.cap_leaves, t.n_leaves = self.n, self.leaf_key.numel(), self.n_leaves
        t.kind, t.key_bits, t.max_level, t.n_grids = self.kind, self.key_bits, self.max_level, len(self.grids)
        t.perm = self.perm.data_ptr()
        t.leaf_start = self.leaf_start.data_ptr()
        t.leaf_key = self.leaf_key.data_ptr()
        t.leaf_level = self.leaf_level.data_ptr()
        t.iperm = self.iperm.data_ptr()
        return t

    @staticmethod
    def _build(x, y, z, grids, n, depth, leaf_cap, device) -> "Tree":
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        iperm = torch.empty(max(n, 1), dtype=torch.int32, device=device)
        leaf_start = torch.empty(n + 1, dtype=torch.int32, device=device)
        leaf_key = torch.empty(max(n, 1), dtype=torch.int64, device=device)
        leaf_level = torch.empty(max(n, 1), dtype=torch.int8, device=device)
        t = L.p2p_tree()
        t.n, t.cap_leaves = n, n
        t.perm, t.leaf_start = perm.data_ptr(), leaf_start.data_ptr()
        t.leaf_key, t.leaf_level = leaf_key.data_ptr(), leaf_level.data_ptr()
        t.iperm = iperm.data_ptr()
        gs, ng = (None, 0)
        if grids is not None:
            gs, _ = grids_struct(grids)
            ng = len(grids)

        def call(ws, nb):
            return L.p2p_build_tree(_ptr(x), _ptr(y), _ptr(z), gs, ng, depth, leaf_cap,
                                    ctypes.byref(t), ws, nb, _stream())
        st, _ = _call(call, device)
        L.check(st)
        nl = int(t.n_leaves)
        return Tree(n=n, n_leaves=nl, kind=int(t.kind), key_bits=int(t.key_bits),
                    max_level=int(t.max_level), perm=perm[:n] if n else perm[:0],
                    leaf_start=leaf_start[: nl + 1], leaf_key=leaf_key[:nl],
                    leaf_level=leaf_level[:nl], iperm=iperm[:n] if n else iperm[:0],
                    grids=list(grids) if grids else [])

    @staticmethod
    def build_particles(x, y, z, depth: int = 20, leaf_cap: int = 64) -> "Tree":
        """Octree over [0,1)^3: uniform of depth `depth` if leaf_cap == 0, else
        adaptive (split iff more than leaf_cap points and level < depth)."""
        for nm, v in (("x", x), ("y", y), ("z", z)):
            _require_device(v, nm, torch.float64)
        return Tree._build(x, y, z, None, x.numel(), depth, leaf_cap, x.device)

    @staticmethod
    def build_grids(grids: Sequence[Grid], device="cuda") -> "Tree":
        """Boxes of 4x4x4 points over one or more regular grids."""
        n = sum(int(g.n_side) ** 3 for g in grids)
        return Tree._build(None, None, None, list(grids), n, 0, 0, torch.device(device))

    def neighbors(self, cap: Optional[int] = None, periodic: bool = False) -> "Nbrs":
        return build_neighbors(self, cap, periodic)


@dataclass
class Nbrs:
    count: int
    nbr_start: torch.Tensor
    nbr_idx: torch.Tensor
    red_entries: int = -1      # S of the redundant layout over these lists (-1: unknown)
    nbr_shift: Optional[torch.Tensor] = None   # int8 image codes of periodic lists

    @property
    def periodic(self) -> bool:
        return self.nbr_shift is not None

    def struct(self) -> L.p2p_nbrs:
        s = L.p2p_nbrs()
        s.cap, s.count = self.nbr_idx.numel(), self.count
        s.nbr_start, s.nbr_idx = self.nbr_start.data_ptr(), self.nbr_idx.data_ptr()
        s.red_entries = self.red_entries
        if self.nbr_shift is not None:
            s.periodic, s.nbr_shift = 1, self.nbr_shift.data_ptr()
        return s


def build_neighbors(tree: Tree, cap: Optional[int] = None, periodic: bool = False,
                    src_tree: Optional[Tree] = None) -> Nbrs:
    """Near lists of every leaf; periodic=True: on the unit torus (particle
    trees), with an image code per entry in nbr_shift.  With src_tree: the
    remote lists of the leaves of `tree` over the leaves of `src_tree`."""
    dev = tree.leaf_start.device
    Lv = tree.n_leaves
    if cap is None:
        cap = (48 if periodic else 32) * max(Lv, 1)
    ts = tree.struct()
    ss = src_tree.struct() if src_tree is not None else None
    for _ in range(2):
        start = torch.empty(Lv + 1, dtype=torch.int64, device=dev)
        idx = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        sh = torch.empty(max(cap, 1), dtype=torch.int8, device=dev) if periodic else None
        s = L.p2p_nbrs()
        s.cap, s.nbr_start, s.nbr_idx = cap, start.data_ptr(), idx.data_ptr()
        if periodic:
            s.periodic, s.nbr_shift = 1, sh.data_ptr()

        def call(ws, nb):
            if ss is not None:
                return L.p2p_build_neighbors_remote(ctypes.byref(ts), ctypes.byref(ss), ctypes.byref(s), ws, nb,
                                                    _stream())
            return L.p2p_build_neighbors(ctypes.byref(ts), ctypes.byref(s), ws, nb, _stream())
        st, _ = _call(call, dev)
        if st == L.P2P_ECAPACITY:
            cap = int(s.count)
            continue
        L.check(st)
        E = int(s.count)
        return Nbrs(count=E, nbr_start=start, nbr_idx=idx[:E], red_entries=int(s.red_entries),
                    nbr_shift=sh[:E] if periodic else None)
    raise L.P2PError(L.P2P_ECAPACITY, "near-list capacity retry failed")


@dataclass
class Redundant:
    count: int
    red_start: torch.Tensor
    red_self: torch.Tensor
    planes: List[Optional[torch.Tensor]]
    nrhs: int
    kind: int
    prec: int
    grain: int = 1                         # 1 box grain; 2 or 4 tiles of grain^3 grid boxes
    red_row: Optional[torch.Tensor] = None  # tile grain: first row of each near-list entry's source

    def struct(self) -> L.p2p_redundant:
        s = L.p2p_redundant()
        s.cap = self.planes[0].shape[0] if self.planes[0] is not None else 0
        s.count = self.count
        s.red_start, s.red_self = self.red_start.data_ptr(), self.red_self.data_ptr()
        for i in range(4):
            s.planes[i] = self.planes[i].data_ptr() if self.planes[i] is not None else None
        s.nrhs, s.kind, s.prec, s.grain = self.nrhs, self.kind, self.prec, self.grain
        s.red_row = self.red_row.data_ptr() if self.red_row is not None else None
        return s


def redundant_entries(tree: Tree, nbrs: Nbrs) -> int:
    """S, the number of entries of the redundant layout (from the near lists,
    else counted on the GPU)."""
    if nbrs.red_entries >= 0:
        return nbrs.red_entries
    return locality(tree, nbrs)["entries"]


def tile_entries(tree: "Tree", grain: int) -> int:
    """S of the tile-grain layout of a grid tree: every tile of grain^3 boxes
    holds the boxes of its window of (grain+2)^3 box cells that exist, 64
    rows each.  The halo size of a tile is the product over the three axes
    of the window's extent inside the grid, so the sum over the tiles of an
    instance is the cube of the sum over one axis (host arithmetic for
    sizing the buffers)."""
    total = 0
    for g in tree.grids:
        nb = g.n_side // 4
        axis = sum(min(o + grain, nb - 1) - max(o - 1, 0) + 1 for o in range(0, nb, grain))
        total += axis ** 3
    return 64 * total


def _alloc_red(tree, kind, prec, S, nrhs, dev):
    if kind == L.P2P_KIND_GRAVITY and prec == L.P2P_FP32_MIXED:
        planes = [torch.empty((max(S, 1), 4), dtype=torch.float32, device=dev), None, None, None]
    elif kind == L.P2P_KIND_GRAVITY:
        planes = [torch.empty((max(S, 1), 4), dtype=torch.float64, device=dev), None, None, None]
    else:
        cd = torch.complex128 if prec == L.P2P_FP64 else torch.complex64
        planes = [torch.empty((max(S, 1), nrhs), dtype=cd, device=dev), None, None, None]
    return planes


def restructure(tree: Tree, nbrs: Nbrs, src: Sequence[Optional[torch.Tensor]], prec="fp64",
                nrhs: int = 1, S: Optional[int] = None, out: Optional[Redundant] = None,
                grain: int = 1) -> Redundant:
    """Restructure into the redundant layout.  Pass `out` (a Redundant of the
    right capacity) to reuse its buffers; pass S to skip the size query.
    grain 1: one segment per target box (leaf); grain 2 or 4 (grid trees):
    one segment per tile of grain^3 boxes."""
    p = PREC[prec]
    dev = tree.leaf_start.device
    kind = L.P2P_KIND_GRAVITY if tree.kind == L.P2P_TREE_PARTICLES else L.P2P_KIND_HELMHOLTZ
    if kind == L.P2P_KIND_GRAVITY:
        if len(src) != 4:
            raise ValueError("gravity sources are x, y, z, m")
        for nm, t in zip("xyzm", src):
            _vec(t, nm, tree.n)
    else:
        if len(src) != 1:
            raise ValueError("Helmholtz sources are one array q")
        _vec(src[0], "q", tree.n * nrhs, torch.complex128 if p == L.P2P_FP64 else torch.complex64)
    if out is None:
        if S is None:
            S = redundant_entries(tree, nbrs) if grain <= 1 else tile_entries(tree, grain)
        out = Redundant(count=0, red_start=torch.empty(tree.n_leaves + 1, dtype=torch.int64, device=dev),
                        red_self=torch.empty(max(tree.n_leaves, 1), dtype=torch.int32, device=dev),
                        planes=_alloc_red(tree, kind, p, S, nrhs, dev), nrhs=nrhs, kind=kind, prec=p,
                        grain=grain,
                        red_row=(torch.empty(max(nbrs.count, 1), dtype=torch.int64, device=dev)
                                 if grain > 1 else None))
    srcs = L.PV4(*[_ptr(t) if t is not None else None for t in list(src) + [None] * (4 - len(src))])
    ts, ns, rs = tree.struct(), nbrs.struct(), out.struct()

    def call(ws, nb):
        return L.p2p_restructure_redundant(ctypes.byref(ts), ctypes.byref(ns), ctypes.byref(srcs),
                                           nrhs, p, ctypes.byref(rs), ws, nb, _stream())
    st, _ = _call(call, dev)
    L.check(st)
    out.count, out.nrhs, out.kind, out.prec = int(rs.count), int(rs.nrhs), int(rs.kind), int(rs.prec)
    return out


def restructure_gravity(tree, nbrs, x, y, z, m, prec="fp64", **kw) -> Redundant:
    return restructure(tree, nbrs, [x, y, z, m], prec=prec, **kw)


def restructure_remote(tree: Tree, src_tree: Tree, nbrs: Nbrs, sx, sy, sz, sm, prec="fp64",
                       out: Optional[Redundant] = None) -> Redundant:
    """Redundant layout of the remote sources (points of `src_tree`) for the
    leaves of `tree`, over remote lists from build_neighbors(src_tree=...)."""
    p = PREC[prec]
    dev = tree.leaf_start.device
    for nm, t in (("sx", sx), ("sy", sy), ("sz", sz), ("sm", sm)):
        _vec(t, nm, src_tree.n)
    if out is None:
        S = nbrs.red_entries
        if S < 0:
            raise ValueError("remote lists without their size")
        out = Redundant(count=0, red_start=torch.empty(tree.n_leaves + 1, dtype=torch.int64, device=dev),
                        red_self=torch.empty(max(tree.n_leaves, 1), dtype=torch.int32, device=dev),
                        planes=_alloc_red(tree, L.P2P_KIND_GRAVITY, p, S, 1, dev), nrhs=1,
                        kind=L.P2P_KIND_GRAVITY, prec=p)
    srcs = L.PV4(*[_ptr(t) for t in (sx, sy, sz, sm)])
    ts, ss, ns, rs = tree.struct(), src_tree.struct(), nbrs.struct(), out.struct()

    def call(ws, nb):
        return L.p2p_restructure_remote(ctypes.byref(ts), ctypes.byref(ss), ctypes.byref(ns),
                                        ctypes.byref(srcs), p, ctypes.byref(rs), ws, nb, _stream())
    st, _ = _call(call, dev)
    L.check(st)
    out.count, out.nrhs, out.kind, out.prec = int(rs.count), int(rs.nrhs), int(rs.kind), int(rs.prec)
    return out


def gravity_remote(tree: Tree, src_tree: Tree, nbrs: Nbrs, eps: float, x, y, z, sx=None, sy=None,
                   sz=None, sm=None, layout="gather", prec="fp64", red: Optional[Redundant] = None, out=None):
    """Remote near-field potential and acceleration of the points of `tree`
    (caller order), added to `out` (zeros when not given).  Returns (phi, ax, ay, az)."""
    dev = tree.leaf_start.device
    for nm, t in (("x", x), ("y", y), ("z", z)):
        _vec(t, nm, tree.n)
    for nm, t in (("sx", sx), ("sy", sy), ("sz", sz), ("sm", sm)):
        _vec(t, nm, src_tree.n, optional=layout == "redundant")
    if out is None:
        out = [torch.zeros(tree.n, dtype=torch.float64, device=dev) for _ in range(4)]
    out = _outs(out, tree.n, dev)
    ts, ss, ns = tree.struct(), src_tree.struct(), nbrs.struct()
    rs = red.struct() if red is not None else None

    def call(ws, nb):
        return L.p2p_eval_gravity_remote(ctypes.byref(ts), ctypes.byref(ss), ctypes.byref(ns),
                                         ctypes.byref(rs) if rs is not None else None,
                                         LAYOUT[layout], PREC[prec], float(eps), _ptr(x), _ptr(y), _ptr(z),
                                         _ptr(sx), _ptr(sy), _ptr(sz), _ptr(sm), *[_ptr(o) for o in out],
                                         ws, nb, _stream())
    st, _ = _call(call, dev)
    L.check(st)
    return tuple(out)


@dataclass
class Interactions:
    """Per-interaction layout (gravity): one record per near-list entry."""
    count: int
    rec_start: torch.Tensor
    rows: torch.Tensor
    target_rows: int
    prec: int

    def struct(self) -> L.p2p_interactions:
        s = L.p2p_interactions()
        s.cap, s.count = self.rows.shape[0], self.count
        s.rec_start = self.rec_start.data_ptr()
        s.planes[0] = self.rows.data_ptr()
        s.target_rows, s.prec = self.target_rows, self.prec
        return s


def restructure_interactions(tree: Tree, nbrs: Nbrs, x, y, z, m, prec="fp64",
                             out: Optional[Interactions] = None) -> Interactions:
    """Restructure into the per-interaction layout (rows float32 [rows, 4]
    for fp32, float64 [rows, 4] for fp64).  Pass `out` to reuse its buffers."""
    p = PREC[prec]
    dev = tree.leaf_start.device
    for nm, t in (("x", x), ("y", y), ("z", z), ("m", m)):
        _vec(t, nm, tree.n)
    E = nbrs.count
    if out is None:
        if nbrs.red_entries >= 0:
            rows = E + 2 * nbrs.red_entries
        else:
            rows = None
        cap = rows if rows is not None else 0
        out = Interactions(count=0, rec_start=torch.empty(E + 1, dtype=torch.int64, device=dev),
                           rows=torch.empty((max(cap, 1), 4), device=dev,
                                            dtype=torch.float32 if p == L.P2P_FP32_MIXED else torch.float64),
                           target_rows=0, prec=p)
    srcs = L.PV4(*[_ptr(t) for t in (x, y, z, m)])
    ts, ns = tree.struct(), nbrs.struct()
    for _ in range(2):
        rs = out.struct()

        def call(ws, nb):
            return L.p2p_restructure_interactions(ctypes.byref(ts), ctypes.byref(ns), ctypes.byref(srcs), p,
                                                  ctypes.byref(rs), ws, nb, _stream())
        st, _ = _call(call, dev)
        if st == L.P2P_ECAPACITY:
            out.rows = torch.empty((int(rs.count), 4), device=dev, dtype=out.rows.dtype)
            continue
        L.check(st)
        out.count, out.target_rows, out.prec = int(rs.count), int(rs.target_rows), int(rs.prec)
        return out
    raise L.P2PError(L.P2P_ECAPACITY, "per-interaction capacity retry failed")


def gravity_interactions(tree: Tree, nbrs: Nbrs, inter: Interactions, eps: float, out=None):
    """Near-field potential and acceleration from the per-interaction layout,
    caller order.  Returns (phi, ax, ay, az)."""
    dev = tree.leaf_start.device
    out = _outs(out, tree.n, dev)
    ts, ns, rs = tree.struct(), nbrs.struct(), inter.struct()

    def call(ws, nb):
        return L.p2p_eval_gravity_interactions(ctypes.byref(ts), ctypes.byref(ns), ctypes.byref(rs),
                                               float(eps), *[_ptr(o) for o in out], ws, nb, _stream())
    st, _ = _call(call, dev)
    L.check(st)
    return tuple(out)


def gravity(tree: Tree, nbrs: Nbrs, eps: float, x=None, y=None, z=None, m=None,
            layout="gather", prec="fp64", red: Optional[Redundant] = None, out=None):
    """Near-field potential and acceleration, caller order.  Returns (phi, ax, ay, az)."""
    dev = tree.leaf_start.device
    n = tree.n
    for nm, t in (("x", x), ("y", y), ("z", z), ("m", m)):
        _vec(t, nm, n, optional=layout == "redundant")
    out = _outs(out, n, dev)
    ts, ns = tree.struct(), nbrs.struct()
    rs = red.struct() if red is not None else None

    def call(ws, nb):
        return L.p2p_eval_gravity(ctypes.byref(ts), ctypes.byref(ns),
                                  ctypes.byref(rs) if rs is not None else None,
                                  LAYOUT[layout], PREC[prec], float(eps), _ptr(x), _ptr(y), _ptr(z),
                                  _ptr(m), *[_ptr(o) for o in out], ws, nb, _stream())
    st, ws = _call(call, dev)
    L.check(st)
    return tuple(out)


def gravity_noalloc(tree: Tree, nbrs: Nbrs, eps: float, x=None, y=None, z=None, m=None,
                    layout="gather", prec="fp64", red: Optional[Redundant] = None, out=None):
    """As gravity(), through p2p_eval_gravity_noalloc: no workspace is
    allocated (the GATHER rows go to the library's static scratch, at most
    2^21 particles).  Calls that overlap on one GPU race on that scratch."""
    dev = tree.leaf_start.device
    n = tree.n
    for nm, t in (("x", x), ("y", y), ("z", z), ("m", m)):
        _vec(t, nm, n, optional=layout == "redundant")
    out = _outs(out, n, dev)
    ts, ns = tree.struct(), nbrs.struct()
    rs = red.struct() if red is not None else None
    st = L.p2p_eval_gravity_noalloc(ctypes.byref(ts), ctypes.byref(ns),
                                           ctypes.byref(rs) if rs is not None else None,
                                           LAYOUT[layout], PREC[prec], float(eps), _ptr(x), _ptr(y), _ptr(z),
                                           _ptr(m), *[_ptr(o) for o in out], _stream())
    L.check(st)
    return tuple(out)


def helmholtz(tree: Tree, nbrs: Nbrs, q: Optional[torch.Tensor] = None, layout="gather",
              prec="fp32", red: Optional[Redundant] = None, nrhs: Optional[int] = None,
              tile: Optional[Sequence[int]] = None, out: Optional[torch.Tensor] = None,
              plan: Optional["HelmholtzPlan"] = None):
    """Near-field Helmholtz on the grids of `tree`.  q, u: [n, nrhs] (or [n])
    complex64 (fp32) or complex128 (fp64), caller order.  With `plan`
    (HelmholtzPlan) the precision, nrhs and tile are the plan's and the call
    does no set-up (p2p_eval_helmholtz_prepared)."""
    dev = tree.leaf_start.device
    if plan is not None:
        prec, nrhs = plan.prec, plan.nrhs
    if nrhs is None:
        nrhs = red.nrhs if red is not None else (1 if q.dim() == 1 else q.shape[1])
    cd = torch.complex128 if PREC[prec] == L.P2P_FP64 else torch.complex64
    _vec(q, "q", tree.n * nrhs, cd, optional=layout == "redundant")
    if out is None:
        shape = (tree.n,) if (q is not None and q.dim() == 1) or (q is None and nrhs == 1) else (tree.n, nrhs)
        out = torch.empty(shape, dtype=cd, device=dev)
    _vec(out, "out", tree.n * nrhs, cd)
    if plan is not None:
        return _helmholtz_prepared(tree, nbrs, plan, q, out, layout, red)
    gs, _ = grids_struct(tree.grids)
    ts, ns = tree.struct(), nbrs.struct()
    rs = red.struct() if red is not None else None
    # (waves per workgroup, workgroups per CU, RHS per wave[, copies of the G blocks])
    tl = (ctypes.c_int32 * 4)(*(tuple(tile) + (1,) * (4 - len(tile)))) if tile is not None else None

    def call(ws, nb):
        return L.p2p_eval_helmholtz(ctypes.byref(ts), ctypes.byref(ns),
                                    ctypes.byref(rs) if rs is not None else None,
                                    LAYOUT[layout], PREC[prec], gs, len(tree.grids), nrhs, _ptr(q),
                                    _ptr(out), tl, ws, nb, _stream())
    st, ws = _call(call, dev)
    L.check(st)
    return out


class HelmholtzPlan:
    """The set-up of the Helmholtz evaluation built once (p2p_helmholtz_prepare):
    parameters and the FP64-built G blocks or tables, in a device buffer
    owned here.  Pass it to helmholtz(..., plan=...)."""

    def __init__(self, tree: Tree, nbrs: Nbrs, prec="fp32", nrhs: int = 1,
                 tile: Optional[Sequence[int]] = None):
        dev = tree.leaf_start.device
        self.prec, self.nrhs = prec, int(nrhs)
        gs, _ = grids_struct(tree.grids)
        ts, ns = tree.struct(), nbrs.struct()
        tl = (ctypes.c_int32 * 4)(*(tuple(tile) + (1,) * (4 - len(tile)))) if tile is not None else None
        p = L.p2p_helmholtz_plan()
        L.check(L.p2p_helmholtz_prepare(ctypes.byref(ts), ctypes.byref(ns), PREC[prec], gs,
                                               len(tree.grids), self.nrhs, tl, ctypes.byref(p), _stream()))
        self.buf = torch.empty(max(int(p.bytes), 1), dtype=torch.uint8, device=dev)
        p.buf = self.buf.data_ptr()
        L.check(L.p2p_helmholtz_prepare(ctypes.byref(ts), ctypes.byref(ns), PREC[prec], gs,
                                               len(tree.grids), self.nrhs, tl, ctypes.byref(p), _stream()))
        self.struct = p


def _helmholtz_prepared(tree, nbrs, plan, q, out, layout, red):
    gs, _ = grids_struct(tree.grids)
    ts, ns = tree.struct(), nbrs.struct()
    rs = red.struct() if red is not None else None

    def call(ws, nb):
        return L.p2p_eval_helmholtz_prepared(ctypes.byref(ts), ctypes.byref(ns),
                                             ctypes.byref(rs) if rs is not None else None, LAYOUT[layout], gs,
                                             len(tree.grids), ctypes.byref(plan.struct), _ptr(q), _ptr(out), ws,
                                             nb, _stream())
    st, _ = _call(call, tree.leaf_start.device)
    L.check(st)
    return out


def gravity_adjoint(tree: Tree, nbrs: Nbrs, eps: float, x, y, z, m, g_phi, g_ax, g_ay, g_az, prec="fp64"):
    """Gradients (g_x, g_y, g_z, g_m) of sum g_phi.phi + g_a.a, tree frozen;
    prec "fp64" or "fp32" (FP32-mixed pair terms)."""
    dev = tree.leaf_start.device
    for nm, t in (("x", x), ("y", y), ("z", z), ("m", m), ("g_phi", g_phi), ("g_ax", g_ax), ("g_ay", g_ay),
                  ("g_az", g_az)):
        _vec(t, nm, tree.n)
    outs = [torch.empty(tree.n, dtype=torch.float64, device=dev) for _ in range(4)]
    fin = L.PV4(*[_ptr(t) for t in (x, y, z, m)])
    gout = L.PV4(*[_ptr(t) for t in (g_phi, g_ax, g_ay, g_az)])
    gin = L.PV4(*[_ptr(t) for t in outs])
    ts, ns = tree.struct(), nbrs.struct()

    def call(ws, nb):
        return L.p2p_adjoint(L.P2P_KIND_GRAVITY, ctypes.byref(ts), ctypes.byref(ns), None,
                             L.P2P_GATHER, PREC[prec], float(eps), None, 0, 1, 0,
                             ctypes.byref(fin), ctypes.byref(gout), ctypes.byref(gin), ws, nb,
                             _stream())
    st, ws = _call(call, dev)
    L.check(st)
    return tuple(outs)


def helmholtz_adjoint(tree: Tree, nbrs: Nbrs, g: torch.Tensor, prec="fp64", conjugate=False):
    """A^T g (conjugate=False) or A^H g = conj(A^T conj(g)) (conjugate=True)."""
    dev = tree.leaf_start.device
    nrhs = 1 if g.dim() == 1 else g.shape[1]
    _vec(g, "g", tree.n * nrhs, torch.complex128 if PREC[prec] == L.P2P_FP64 else torch.complex64)
    out = torch.empty_like(g)
    gs, _ = grids_struct(tree.grids)
    gout = L.PV4(_ptr(g), None, None, None)
    gin = L.PV4(_ptr(out), None, None, None)
    ts, ns = tree.struct(), nbrs.struct()

    def call(ws, nb):
        return L.p2p_adjoint(L.P2P_KIND_HELMHOLTZ, ctypes.byref(ts), ctypes.byref(ns), None,
                             L.P2P_GATHER, PREC[prec], 0.0, gs, len(tree.grids), nrhs,
                             1 if conjugate else 0, None, ctypes.byref(gout), ctypes.byref(gin),
                             ws, nb, _stream())
    st, ws = _call(call, dev)
    L.check(st)
    return out


def locality(tree: Tree, nbrs: Nbrs, red: Optional[Redundant] = None, bytes_per_entry=32.0,
             cache_bytes=32.0 * 2 ** 20) -> dict:
    """Locality metric (Definition 1, Formulas (10)/(11)) plus exact pair and entry counts."""
    dev = tree.leaf_start.device
    ts, ns = tree.struct(), nbrs.struct()
    rs = red.struct() if red is not None else None
    out = L.p2p_locality_t()

    def call(ws, nb):
        return L.p2p_locality(ctypes.byref(ts), ctypes.byref(ns),
                              ctypes.byref(rs) if rs is not None else None, float(bytes_per_entry),
                              float(cache_bytes), ctypes.byref(out), ws, nb, _stream())
    st, _ = _call(call, dev)
    L.check(st)
    return {f: getattr(out, f) for f, _ in L.p2p_locality_t._fields_}


class Graph:
    """Library calls recorded once into a HIP graph (through
    torch.cuda.CUDAGraph) and replayed with one launch each time, which
    removes the host launch gaps between the short kernels of a step.  Every
    replay runs the kernels recorded at capture on the same arrays: the tree,
    lists, layouts, inputs and outputs the calls used must stay alive and in
    place, and new input values are written into those arrays.  Workspaces
    taken during capture stay reserved for the graph.  Calls that read back,
    synchronise or copy from host memory raise P2PError (P2P_EUNSUPPORTED)
    during capture."""

    def __init__(self, fn, warmup: int = 1):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                fn()
        torch.cuda.current_stream().wait_stream(side)
        self._graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self._graph):
            fn()

    def replay(self) -> None:
        self._graph.replay()

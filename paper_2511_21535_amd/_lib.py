"""ctypes binding of libp2p (include/p2p.h), argument marshalling only.

Every function here has the name of the C entry point it calls and takes the
same arguments.  Loading fails loudly if the built library is missing: there
is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libp2p.so")

P2P_OK, P2P_EINVAL, P2P_EDOMAIN, P2P_ECAPACITY, P2P_EHIP, P2P_EUNSUPPORTED = range(6)
P2P_GATHER, P2P_REDUNDANT = 0, 1
P2P_FP64, P2P_FP32_MIXED, P2P_FP32 = 0, 1, 2
P2P_TREE_PARTICLES, P2P_TREE_GRIDS = 0, 1
P2P_KIND_GRAVITY, P2P_KIND_HELMHOLTZ = 0, 1

STATUS_NAMES = {0: "P2P_OK", 1: "P2P_EINVAL", 2: "P2P_EDOMAIN", 3: "P2P_ECAPACITY",
                4: "P2P_EHIP", 5: "P2P_EUNSUPPORTED"}

EXPORTED = ["p2p_build_tree", "p2p_build_neighbors", "p2p_restructure_redundant",
            "p2p_eval_gravity", "p2p_eval_helmholtz", "p2p_adjoint", "p2p_locality",
            "p2p_restructure_interactions", "p2p_eval_gravity_interactions",
            "p2p_build_neighbors_remote", "p2p_restructure_remote", "p2p_eval_gravity_remote",
            "p2p_eval_gravity_noalloc", "p2p_helmholtz_prepare", "p2p_eval_helmholtz_prepared",
            "p2p_last_error", "p2p_version"]


class p2p_grid(ctypes.Structure):
    _fields_ = [("n_side", ctypes.c_int32), ("reserved", ctypes.c_int32), ("h", ctypes.c_double),
                ("k", ctypes.c_double), ("point_off", ctypes.c_int64)]


class p2p_tree(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("cap_leaves", ctypes.c_int64), ("n_leaves", ctypes.c_int64),
                ("kind", ctypes.c_int32), ("key_bits", ctypes.c_int32),
                ("max_level", ctypes.c_int32), ("n_grids", ctypes.c_int32),
                ("perm", ctypes.c_void_p), ("leaf_start", ctypes.c_void_p),
                ("leaf_key", ctypes.c_void_p), ("leaf_level", ctypes.c_void_p),
                ("iperm", ctypes.c_void_p)]


class p2p_nbrs(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64), ("count", ctypes.c_int64),
                ("nbr_start", ctypes.c_void_p), ("nbr_idx", ctypes.c_void_p),
                ("red_entries", ctypes.c_int64), ("periodic", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("nbr_shift", ctypes.c_void_p)]


class p2p_redundant(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64), ("count", ctypes.c_int64),
                ("red_start", ctypes.c_void_p), ("red_self", ctypes.c_void_p),
                ("planes", ctypes.c_void_p * 4), ("nrhs", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("grain", ctypes.c_int32), ("red_row", ctypes.c_void_p)]


class p2p_interactions(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int64), ("count", ctypes.c_int64), ("rec_start", ctypes.c_void_p),
                ("planes", ctypes.c_void_p * 1), ("target_rows", ctypes.c_int64),
                ("prec", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class p2p_locality_t(ctypes.Structure):
    _fields_ = [("d_mean", ctypes.c_double), ("v_gather", ctypes.c_double),
                ("v_red", ctypes.c_double), ("d_ratio", ctypes.c_double),
                ("v_ratio", ctypes.c_double), ("locality", ctypes.c_double),
                ("pairs", ctypes.c_int64), ("entries", ctypes.c_int64)]


class p2p_helmholtz_plan(ctypes.Structure):
    _fields_ = [("buf", ctypes.c_void_p), ("bytes", ctypes.c_size_t), ("prec", ctypes.c_int32),
                ("nrhs", ctypes.c_int32), ("tile", ctypes.c_int32 * 4), ("tiled", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("fingerprint", ctypes.c_uint64)]


_lib = None
V = ctypes.c_void_p
PV4 = ctypes.c_void_p * 4
SZ = ctypes.POINTER(ctypes.c_size_t)


def load():
    """Load libp2p.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libp2p.so not found at {LIB_PATH}: build it with "
                           "`python -m paper_2511_21535_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    I32, I64, F64, st = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    lib.p2p_build_tree.restype = st
    lib.p2p_build_tree.argtypes = [V, V, V, ctypes.POINTER(p2p_grid), I32, I32, I32,
                                   ctypes.POINTER(p2p_tree), V, SZ, V]
    lib.p2p_build_neighbors.restype = st
    lib.p2p_build_neighbors.argtypes = [ctypes.POINTER(p2p_tree), ctypes.POINTER(p2p_nbrs), V, SZ, V]
    lib.p2p_restructure_redundant.restype = st
    lib.p2p_restructure_redundant.argtypes = [ctypes.POINTER(p2p_tree), ctypes.POINTER(p2p_nbrs),
                                              ctypes.POINTER(PV4), I32, I32,
                                              ctypes.POINTER(p2p_redundant), V, SZ, V]
    lib.p2p_eval_gravity.restype = st
    lib.p2p_eval_gravity.argtypes = [ctypes.POINTER(p2p_tree), ctypes.POINTER(p2p_nbrs),
                                     ctypes.POINTER(p2p_redundant), I32, I32, F64,
                                     V, V, V, V, V, V, V, V, V, SZ, V]
    lib.p2p_eval_helmholtz.restype = st
    lib.p2p_eval_helmholtz.argtypes = [ctypes.POINTER(p2p_tree), ctypes.POINTER(p2p_nbrs),
                                       ctypes.POINTER(p2p_redundant), I32, I32,
                                       ctypes.POINTER(p2p_grid), I32, I32, V, V,
                                       ctypes.POINTER(ctypes.c_int32), V, SZ, V]
    lib.p2p_adjoint.restype = st
    lib.p2p_adjoint.argtypes = [I32, ctypes.POINTER(p2p_tree), ctypes.POINTER(p2p_nbrs),
                                ctypes.POINTER(p2p_redundant), I32, I32, F64,
                                ctypes.POINTER(p2p_grid), I32, I32, I32,
                                ctypes.POINTER(PV4), ctypes.POINTER(PV4), ctypes.POINTER(PV4),
                                V, SZ, V]
    lib.p2p_restructure_interactions.restype = st
    lib.p2p_restructure_interactions.argtypes = [ctypes.POINTER(p2p_tree), ctypes.POINTER(p2p_nbrs),
                                                 ctypes.POINTER(PV4), I32,
                                                 ctypes.POINTER(p2p_interactions), V, SZ, V]
    lib.p2p_eval_gravity_interactions.restype = st
    lib.p2p_eval_gravity_interactions.argtypes = [ctypes.POINTER(p2p_tree), ctypes.POINTER(p2p_nbrs),
                                                  ctypes.POINTER(p2p_interactions), F64,
                                                  V, V, V, V, V, SZ, V]
    T, N, R = ctypes.POINTER(p2p_tree), ctypes.POINTER(p2p_nbrs), ctypes.POINTER(p2p_redundant)
    lib.p2p_build_neighbors_remote.restype = st
    lib.p2p_build_neighbors_remote.argtypes = [T, T, N, V, SZ, V]
    lib.p2p_restructure_remote.restype = st
    lib.p2p_restructure_remote.argtypes = [T, T, N, ctypes.POINTER(PV4), I32, R, V, SZ, V]
    lib.p2p_eval_gravity_remote.restype = st
    lib.p2p_eval_gravity_remote.argtypes = [T, T, N, R, I32, I32, F64] + [V] * 11 + [V, SZ, V]
    lib.p2p_eval_gravity_noalloc.restype = st
    lib.p2p_eval_gravity_noalloc.argtypes = [T, N, R, I32, I32, F64] + [V] * 8 + [V]
    HP, GP = ctypes.POINTER(p2p_helmholtz_plan), ctypes.POINTER(p2p_grid)
    lib.p2p_helmholtz_prepare.restype = st
    lib.p2p_helmholtz_prepare.argtypes = [T, N, I32, GP, I32, I32, ctypes.POINTER(ctypes.c_int32), HP, V]
    lib.p2p_eval_helmholtz_prepared.restype = st
    lib.p2p_eval_helmholtz_prepared.argtypes = [T, N, R, I32, GP, I32, HP, V, V, V, SZ, V]
    lib.p2p_locality.restype = st
    lib.p2p_locality.argtypes = [ctypes.POINTER(p2p_tree), ctypes.POINTER(p2p_nbrs),
                                 ctypes.POINTER(p2p_redundant), F64, F64,
                                 ctypes.POINTER(p2p_locality_t), V, SZ, V]
    lib.p2p_last_error.restype = ctypes.c_char_p
    lib.p2p_last_error.argtypes = []
    lib.p2p_version.restype = ctypes.c_char_p
    lib.p2p_version.argtypes = []
    _lib = lib
    return lib


class P2PError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def last_error() -> str:
    return load().p2p_last_error().decode()


def check(status: int):
    if status != P2P_OK:
        raise P2PError(status, last_error())
    return status


# Same names as the C entry points; arguments passed through unchanged.
def p2p_build_tree(*args):
    return load().p2p_build_tree(*args)


def p2p_build_neighbors(*args):
    return load().p2p_build_neighbors(*args)


def p2p_restructure_redundant(*args):
    return load().p2p_restructure_redundant(*args)


def p2p_eval_gravity(*args):
    return load().p2p_eval_gravity(*args)


def p2p_eval_helmholtz(*args):
    return load().p2p_eval_helmholtz(*args)


def p2p_adjoint(*args):
    return load().p2p_adjoint(*args)


def p2p_restructure_interactions(*args):
    return load().p2p_restructure_interactions(*args)


def p2p_eval_gravity_interactions(*args):
    return load().p2p_eval_gravity_interactions(*args)


def p2p_build_neighbors_remote(*args):
    return load().p2p_build_neighbors_remote(*args)


def p2p_restructure_remote(*args):
    return load().p2p_restructure_remote(*args)


def p2p_eval_gravity_remote(*args):
    return load().p2p_eval_gravity_remote(*args)


def p2p_eval_gravity_noalloc(*args):
    return load().p2p_eval_gravity_noalloc(*args)


def p2p_helmholtz_prepare(*args):
    return load().p2p_helmholtz_prepare(*args)


def p2p_eval_helmholtz_prepared(*args):
    return load().p2p_eval_helmholtz_prepared(*args)


def p2p_locality(*args):
    return load().p2p_locality(*args)


def p2p_last_error():
    return load().p2p_last_error().decode()


def p2p_version():
    return load().p2p_version().decode()

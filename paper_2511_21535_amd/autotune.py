"""Autotuner for the launch shape of the multi-RHS Helmholtz matrix-core kernel.

Candidates are (waves per workgroup, workgroups per CU, right-hand sides per
wave); the best of them is then tried with 2, 4 and 8 copies of the G blocks
in memory (the pattern redundancy factor), and the fewest copies within 2% of
the fastest time are kept.  Each candidate is timed on the
actual problem with HIP events (one warm-up, then the median of `reps` calls)
and the fastest is cached in a JSON file keyed by device name, grid sizes,
nrhs and layout.  The cache path is
$P2P_AUTOTUNE_CACHE, else ~/.cache/p2p_mi355x_autotune.json.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Optional, Sequence, Tuple

import torch

from . import api

CANDIDATES = [(w, c, r) for w in (1, 2, 4) for c in (1, 2, 3, 4, 6, 8) for r in (32, 64)]
# copies of the G blocks (the pattern redundancy factor), tuned on the best shape
COPIES = (1, 2, 4, 8)
# a copy count is kept over a smaller one only if it is faster by more than this
COPY_MARGIN = 0.02


def cache_path() -> str:
    return os.environ.get("P2P_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "p2p_mi355x_autotune.json"))


def problem_key(tree: api.Tree, nrhs: int, layout: str, prec: str = "fp32") -> str:
    dev = torch.cuda.get_device_name(tree.leaf_start.device)
    sizes = ",".join(str(g.n_side) for g in tree.grids)
    h = hashlib.sha1(sizes.encode()).hexdigest()[:16]
    return f"{dev}|grids={len(tree.grids)}:{h}|nrhs={nrhs}|{layout}|{prec}"


def _load_cache() -> Dict[str, dict]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c: Dict[str, dict]) -> None:
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def time_call(fn, reps: int = 3) -> float:
    """Median milliseconds of fn() over `reps` calls after one warm-up."""
    fn()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    return ts[len(ts) // 2]


def pick_copies(timings: Dict[str, float], shape: Sequence[int], copies: Sequence[int] = COPIES
                ) -> Tuple[int, int, int, int]:
    """The tile for the launch shape `shape`: more copies of the G blocks cost
    memory and HBM traffic (each copy misses in L2 on its own), so the fewest
    copies whose time is within COPY_MARGIN of the fastest timing are kept."""
    best_ms = min(timings.values())
    for c in sorted(copies):
        k = str(list(shape) + [c])
        if k in timings and timings[k] <= best_ms * (1.0 + COPY_MARGIN):
            return tuple(shape) + (c,)
    return tuple(json.loads(min(timings, key=timings.get)))


def tune_helmholtz(tree: api.Tree, nbrs: api.Nbrs, q: Optional[torch.Tensor] = None,
                   red: Optional[api.Redundant] = None, layout: str = "gather",
                   candidates: Sequence[Tuple[int, int, int]] = CANDIDATES, reps: int = 3,
                   use_cache: bool = True, copies: Sequence[int] = COPIES, prec: str = "fp32"
                   ) -> Tuple[Tuple[int, int, int, int], Dict[str, float]]:
    """Pick the fastest launch shape, then the number of copies of the G
    blocks; returns (tile, timings), tile = (waves per workgroup, workgroups
    per CU, RHS per wave, copies).  prec: "fp32" (FP64 per-target sums of the
    per-box partial products) or "fp32_plain"."""
    nrhs = red.nrhs if red is not None else q.shape[1]
    key = problem_key(tree, nrhs, layout, prec)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        e = cache[key]
        return tuple(e["tile"]), e.get("ms", {})
    out = torch.empty((tree.n, nrhs), dtype=torch.complex64, device=tree.leaf_start.device)
    timings = {}

    def run(cand):
        fn = lambda: api.helmholtz(tree, nbrs, q, layout=layout, prec=prec, red=red, nrhs=nrhs,
                                   tile=cand, out=out)
        timings[str(list(cand))] = time_call(fn, reps)

    # launch shape first (one copy of the G blocks), then the number of copies
    for cand in candidates:
        if nrhs % cand[2] == 0:
            run(tuple(cand)[:3] + (1,))
    shape = json.loads(min(timings, key=timings.get))[:3]
    for c in copies:
        if c != 1:
            run(tuple(shape) + (c,))
    tile = pick_copies(timings, shape, copies)
    if use_cache:
        cache = _load_cache()
        cache[key] = {"tile": list(tile), "ms": timings}
        _save_cache(cache)
    return tile, timings


# redundancy grains: one segment per box (1), or per tile of 2^3 or 4^3 boxes
GRAINS = (1, 2, 4)


def tune_grain(tree: api.Tree, nbrs: api.Nbrs, q: torch.Tensor, nrhs: int, prec: str = "fp32",
               tile: Optional[Sequence[int]] = None, grains: Sequence[int] = GRAINS, reps: int = 3
               ) -> Tuple[int, Dict[int, Dict[str, float]]]:
    """The redundancy grain of a grid batch (Sec. 3.5: per-block redundancy
    for dense regular data): for each grain, the restructure and the
    redundant evaluation are timed on the actual problem (median of `reps`
    after a warm-up), each layout allocated, timed and freed in turn.
    Returns (grain with the least restructure + evaluation time, timings in
    ms per grain)."""
    out = torch.empty_like(q)
    res = {}
    for g in grains:
        red = api.restructure(tree, nbrs, [q], prec=prec, nrhs=nrhs, grain=g)
        t_res = time_call(lambda: api.restructure(tree, nbrs, [q], prec=prec, nrhs=nrhs, out=red), reps)
        t_ev = time_call(lambda: api.helmholtz(tree, nbrs, None, layout="redundant", prec=prec, red=red,
                                               nrhs=nrhs, tile=tile, out=out), reps)
        res[g] = {"restructure_ms": t_res, "eval_redundant_ms": t_ev, "entries": red.count}
        del red
        torch.cuda.empty_cache()
    best = min(res, key=lambda g: res[g]["restructure_ms"] + res[g]["eval_redundant_ms"])
    return best, res

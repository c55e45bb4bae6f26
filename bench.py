"""Benchmark: near-field pair-interactions/s, redundant vs gather layout
(restructure included), on one MI355X.

Workload (the irregular gravity case): 2^21 particles from a mixture of 8
Plummer spheres, adaptive octree with leaf cap 64, Plummer softening 1e-3,
FP32-mixed pair arithmetic.  One step is one pass of the whole path over the
resident inputs: tree binning, near lists, restructure to the redundant
layout, redundant evaluation, gather evaluation (the update into caller order
is fused into both evaluations).  Every sub-step is timed with HIP events on
the stream the library launches on.

value = pairs / (restructure + redundant evaluation), over the K timed steps.
The line also carries the rate without the restructure, the gather rate, the
sub-step times, the Locality metric, the roofline of the dominant kernel
(the redundant evaluation) and the FP64 CPU oracle timed on a sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "gravity_plummer_2m"
METRIC = "near-field pair-interactions/s, redundant vs gather layout (incl. restructure)"

# Roofline of the redundant evaluation (VALU-bound): minimal VALU issue slots
# per FP32-mixed pair: 3 FP64 differences, 3 conversions to FP32, 3 FMA for
# r^2 + eps^2, 1 quarter-rate rsqrt (4 slots), 3 multiplies (w^2, m w,
# m w^3), 1 add (phi) and 3 FMA (a).
SLOTS_PER_PAIR = 3 + 3 + 3 + 4 + 3 + 1 + 3          # = 20
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = VALU lane-slots per second
VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9               # = 3.93e13


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-leaves", type=int, default=0,
                    help="target leaves in the CPU oracle sample (0 = all)")
    return ap.parse_args()


def cpu_baseline(x, y, z, m, w, n_leaves_sample, min_seconds=10.0, max_reps=8):
    """The FP64 oracle, as it stands, on target leaves of the same workload
    (all of them by default): pairs evaluated per second of oracle evaluation
    time, the evaluation repeated until about `min_seconds` have passed
    (median of the repeats).  The oracle's tree and brute-force near lists
    are built first and not timed."""
    import oracle
    t0 = time.perf_counter()
    ot = oracle.build_tree_particles(x, y, z, depth=w["depth"], leaf_cap=w["leaf_cap"])
    t_tree = time.perf_counter() - t0
    k = ot.n_leaves if n_leaves_sample <= 0 else min(n_leaves_sample, ot.n_leaves)
    if k == ot.n_leaves:
        sel = np.arange(k, dtype=np.int32)
        what = f"all {k} target leaves"
    else:
        rng = np.random.default_rng(123)
        sel = np.sort(rng.choice(ot.n_leaves, k, replace=False)).astype(np.int32)
        what = f"{k} of {ot.n_leaves} target leaves drawn uniformly (seed 123)"
    ss, si = oracle.neighbors(ot, sel)
    occ = np.diff(ot.leaf_start).astype(np.int64)
    seg = np.add.reduceat(occ[si], ss[:-1])
    pairs = int((occ[sel] * seg).sum() - occ[sel].sum())
    times = []
    while len(times) < max_reps and (sum(times) < min_seconds or len(times) < 3):
        t0 = time.perf_counter()
        oracle.gravity_leaves(x, y, z, m, w["eps"], ot, sel, ss, si)
        times.append(time.perf_counter() - t0)
    t_eval = float(np.median(times))
    return {"value": pairs / t_eval, "unit": "pair-interactions/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{what}, {pairs} pairs, FP64 plain loops, median of {len(times)} evaluations "
                      f"of {t_eval:.2f} s (oracle tree build {t_tree:.2f} s and near lists not counted)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the near-field path is built and measured for a single MI355X.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2511_21535_amd import api
    from paper_2511_21535_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = W.WORKLOADS[WORKLOAD]
    x, y, z, m = W.particles(WORKLOAD)
    gx, gy, gz, gm = (torch.as_tensor(v, device=dev) for v in (x, y, z, m))
    eps, prec = w["eps"], "fp32"
    n = x.shape[0]

    # sizes (one untimed pass): leaves, near entries, redundant entries, pairs
    tree = api.Tree.build_particles(gx, gy, gz, depth=w["depth"], leaf_cap=w["leaf_cap"])
    nbrs = tree.neighbors()
    loc = api.locality(tree, nbrs, bytes_per_entry=28.0, cache_bytes=32.0 * 2 ** 20)
    S, pairs = int(loc["entries"]), int(loc["pairs"])
    red = api.restructure_gravity(tree, nbrs, gx, gy, gz, gm, prec=prec, S=S)
    outs = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4)]

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def step():
        e = [ev() for _ in range(6)]
        e[0].record()
        t = api.Tree.build_particles(gx, gy, gz, depth=w["depth"], leaf_cap=w["leaf_cap"])
        e[1].record()
        nb = t.neighbors(cap=nbrs.count)
        e[2].record()
        r = api.restructure_gravity(t, nb, gx, gy, gz, gm, prec=prec, out=red)
        e[3].record()
        api.gravity(t, nb, eps, layout="redundant", prec=prec, red=r, out=outs)
        e[4].record()
        api.gravity(t, nb, eps, x=gx, y=gy, z=gz, m=gm, layout="gather", prec=prec, out=outs)
        e[5].record()
        return e

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([[a.elapsed_time(b) for a, b in zip(e[:-1], e[1:])] for e in evs])  # [K, 5]
    t_tree, t_nbr, t_res, t_red, t_gat = ms.sum(0) / 1e3   # seconds over K steps
    K = args.steps
    value = pairs * K / (t_res + t_red)
    rate_red = pairs * K / t_red
    rate_gat = pairs * K / t_gat
    avg_red = t_red / K
    achieved = pairs * SLOTS_PER_PAIR / avg_red / 1e12
    peak = VALU_PEAK_SLOTS / 1e12
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": "gravity_plummer_2m: 2^21 particles, 8 Plummer spheres (scale radii "
                        "0.01-0.1), adaptive octree leaf cap 64, eps 1e-3, FP32-mixed",
            "n": n, "leaves": tree.n_leaves, "max_level": tree.max_level,
            "near_entries": nbrs.count, "redundant_entries": S, "pairs": pairs,
            "parallelism": "single GPU",
        },
        "rates": {
            "redundant_incl_restructure": value,
            "redundant_excl_restructure": rate_red,
            "gather": rate_gat,
            "speedup_redundant_vs_gather_incl_restructure": value / rate_gat,
            "speedup_redundant_vs_gather_kernel_only": rate_red / rate_gat,
        },
        "ms": {"tree": t_tree / K * 1e3, "neighbors": t_nbr / K * 1e3, "restructure": t_res / K * 1e3,
               "eval_redundant": t_red / K * 1e3, "eval_gather": t_gat / K * 1e3},
        "locality": {k: loc[k] for k in ("d_mean", "d_ratio", "v_ratio", "locality")},
        "roofline": {"bound": "alu", "kernel": "k_gravity<mixed, redundant>",
                     "achieved": achieved, "peak": peak, "unit": "T VALU lane-slots/s",
                     "frac": achieved / peak, "traffic": None,
                     "algorithmic_per_pair": SLOTS_PER_PAIR},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(x, y, z, m, w, args.cpu_leaves)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

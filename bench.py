"""Benchmark: near-field pair-interactions/s, redundant vs gather layout
(restructure included), on one MI355X.

Default workload (the largest configuration): 128 independent grid instances
of edge 16..48 points (leaf boxes of 4^3 points, k at 10 points per
wavelength), 64 complex right-hand sides each, evaluated in one persistent
launch on the FP32 matrix cores with autotuned tiles.  One step is one pass of
the whole path over the resident inputs: tree binning, near lists,
restructure to the redundant layout, redundant evaluation, gather evaluation
(the update into caller order is fused into both evaluations).  Every
sub-step is timed with HIP events on the stream the library launches on.

value = work / (restructure + redundant evaluation), over the K timed steps
(work = pairs x right-hand sides).  The line also carries the rate without
the restructure, the gather rate, the sub-step times, the Locality metric with
the paper's speedup model evaluated on the measured times (Sec. 3.2-3.4), the
roofline of the dominant kernel, the error of every result against the FP64
oracle on sampled targets, and the FP64 CPU oracle timed on a sample of the
workload.

The default run also measures the irregular gravity case in the same way and
nests its line under "gravity_plummer_2m": 2^21 particles from a mixture of 8
Plummer spheres, adaptive octree with leaf cap 64, Plummer softening 1e-3,
FP32-mixed pair arithmetic.  Gravity lines also time the per-interaction
layout (one record per near-list entry, results per record summed
afterwards) on the same tree and lists, the same tree on the unit torus
(periodic images), and the local, remote and periodic interaction types of
one half of the domain, all outside the timed steps.

--workload selects one configuration on its own:
  helmholtz_batched_128x64  (default) 128 grids 16^3..48^3, 64 RHS, FP32 matrix cores
  gravity_plummer_2m        2^21 Plummer-mixture particles, leaf cap 64, FP32-mixed
  gravity_uniform_4096      4096 uniform particles, uniform depth 3, FP64
  helmholtz_grid_64         64^3 grid, 1 RHS, FP32 matrix cores (target boxes as columns)
  adjoint_gravity_256k      2^18 Plummer particles, forward + adjoint, FP64 and FP32-mixed
  adjoint_helmholtz_48      48^3 grid, forward + adjoint (A^T g), FP64

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu] [--no-nested]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2511_21535_amd import speedup_model  # noqa: E402  (host arithmetic only)

DEFAULT_WORKLOAD = "helmholtz_batched_128x64"
NESTED_WORKLOAD = "gravity_plummer_2m"
METRIC = "near-field pair-interactions/s, redundant vs gather layout (incl. restructure)"

# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = VALU lane-slots per second
VALU_PEAK_SLOTS = 256 * 4 * 16 * 2.4e9               # = 3.93e13
# Minimal VALU issue slots per FP32-mixed gravity pair, coordinates already
# relative to the target leaf's centre (the double subtraction of the offset
# is per (target leaf, source), not per pair): 3 FP32 differences, 3 FMA for
# r^2 + eps^2, 1 v_rsq_f32 (2 slots: it issues at half rate, measured by
# `bench.py --peaks`), 3 multiplies (w^2, m w, m w^3), 1 FMA (phi) and 3 FMA
# (a).
SLOTS_PER_PAIR_MIXED = 3 + 3 + 2 + 3 + 1 + 3        # = 15
# FP64 gravity pair: the instructions hipcc emits per pair, each taken as one
# slot: 3 differences, 3 FMA for r^2 + eps^2, 3 multiplies, 1 FMA (phi),
# 3 FMA (a), and 6 for the reciprocal square root (v_rsq_f64 and one
# third-order refinement step to full precision).
SLOTS_PER_PAIR_FP64 = 3 + 3 + 3 + 1 + 3 + 6         # = 19
# Gravity adjoint per pair, the VALU instructions hipcc emits in the pair
# loop without its loop control: FP64 33 arithmetic + 6 for the reciprocal
# square root (as in the forward count); FP32-mixed 34, with v_rsq_f32 at
# half rate (one more slot).  The term w^3 (m_j ga_k - m_k ga_j) is summed as
# two running sums (m_j sum w^3 ga_k - ga_j sum w^3 m_k), which took 8 of the
# 41 and 42 instructions a per-pair difference needed.
SLOTS_PER_PAIR_ADJ_FP64 = 33 + 6                     # = 39
SLOTS_PER_PAIR_ADJ_MIXED = 34 + 1                    # = 35
# FP32 vector FMA without packed issue: 256 CUs x 64 lanes x 2 flop x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12  # = 78.6
FP32_MFMA_PEAK_TFLOPS = 157.3                        # dense FP32 matrix (published)
FP64_VALU_PEAK_TFLOPS = 78.6                         # FP64 vector (published)
FP64_MFMA_PEAK_TFLOPS = 78.6                         # dense FP64 matrix (published)
CACHE_BYTES = 32.0 * 2 ** 20                         # C of the Locality metric: 8 XCDs x 4 MB L2


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the timing of the CPU oracle (the error against it is still taken, on a "
                         "smaller sample)")
    ap.add_argument("--no-nested", action="store_true",
                    help="with the default workload, skip the nested gravity_plummer_2m line")
    ap.add_argument("--cpu-leaves", type=int, default=0,
                    help="target leaves in the CPU oracle sample (0 = all)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain device copies of 1 GiB, the reference for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters, and print the copy and fill rates")
    ap.add_argument("--peaks", action="store_true",
                    help="only run the microbenchmarks of libp2p_peaks (FP32 FMA issue, v_rsq_f32 issue, "
                         "FP32 matrix cores) and print the measured rates")
    return ap.parse_args()


def copy_calibration():
    """Plain device-to-device copies of 2^30 bytes (3, then 5 timed), the
    reference for scaling the FETCH_SIZE / WRITE_SIZE counters; also the copy
    and fill rates of that size (HIP events)."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    ev = _events(3)
    ev[0].record()
    for _ in range(5):
        b.copy_(a)
    ev[1].record()
    for _ in range(5):
        b.fill_(1.0)
    ev[2].record()
    torch.cuda.synchronize()
    nb = a.numel() * 4
    print(json.dumps({"copy_calibration_bytes": nb, "reps": 3,
                      "copy_GBps_read_plus_write": 2 * nb * 5 / ev[0].elapsed_time(ev[1]) / 1e6,
                      "fill_GBps_write": nb * 5 / ev[1].elapsed_time(ev[2]) / 1e6}), flush=True)


PEAK_BLOCKS = 8192          # 256-thread workgroups per microbenchmark launch (4 per CU slot, 4 rounds)
PEAK_ITERS = {"fma": 1000, "rsq": 1000, "mfma": 500}


def peaks():
    """Measured denominators beside the published peaks: an FP32 FMA loop
    (lane-slots/s), a v_rsq_f32 loop (its cost in lane-slots is the FMA rate
    over its rate) and a v_mfma_f32_16x16x4f32 loop (TFLOP/s), each launch
    timed with HIP events on the stream it runs on (median of 5, after 2)."""
    import ctypes
    import torch
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2511_21535_amd", "libp2p_peaks.so"))
    out = torch.empty(PEAK_BLOCKS * 256, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    res = {}
    for name, fn in (("fma", lib.p2pk_valu_fma), ("rsq", lib.p2pk_valu_rsq), ("mfma", lib.p2pk_mfma_f32)):
        fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p]
        fn.restype = ctypes.c_int
        it = PEAK_ITERS[name]
        times = []
        for rep in range(7):
            ev = _events(2)
            ev[0].record()
            rc = fn(ctypes.c_void_p(out.data_ptr()), PEAK_BLOCKS, it, ctypes.c_void_p(stream))
            ev[1].record()
            if rc != 0:
                raise RuntimeError(f"p2pk {name}: launch returned {rc}")
            torch.cuda.synchronize()
            if rep >= 2:
                times.append(ev[0].elapsed_time(ev[1]) / 1e3)
        t = float(np.median(times))
        threads = PEAK_BLOCKS * 256
        if name == "fma":
            res["valu_fma_T_lane_slots_per_s"] = threads * it * 128 / t / 1e12
        elif name == "rsq":
            res["valu_rsq_T_per_s"] = threads * it * 64 / t / 1e12
        else:
            res["mfma_f32_TFLOPs"] = (threads // 64) * it * 32 * 2048 / t / 1e12
        res[f"{name}_ms"] = t * 1e3
    res["rsq_lane_slots"] = res["valu_fma_T_lane_slots_per_s"] / res["valu_rsq_T_per_s"]
    res["published"] = {"valu_T_lane_slots_per_s": VALU_PEAK_SLOTS / 1e12, "mfma_f32_TFLOPs": FP32_MFMA_PEAK_TFLOPS}
    print(json.dumps(res), flush=True)


def pmc_traffic(kernel, workload, source):
    """HBM bytes per launch of `kernel` on `workload`, from the FETCH_SIZE and
    WRITE_SIZE counter summary kept in profiles/<kernel>_<workload>_hbm_counters.md,
    each counter scaled by what it reads for a plain copy of known size.  The
    summary records the SHA-256 of the kernel's source file when the counters
    were taken; if that file has changed since, or there is no summary, the
    traffic is unknown (None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_counters.md")
    try:
        rec = next(json.loads(l.split("record:", 1)[1]) for l in open(path) if l.startswith("record:"))
    except (OSError, StopIteration, ValueError):
        return None
    with open(os.path.join(ROOT, "paper_2511_21535_amd", "csrc", source), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    return {"bytes": rec["fetch_kib"] * 1024 * rec["fetch_scale"] + rec["write_kib"] * 1024 * rec["write_scale"],
            "read_bytes": rec["fetch_kib"] * 1024 * rec["fetch_scale"],
            "write_bytes": rec["write_kib"] * 1024 * rec["write_scale"]}


def measured_peaks():
    """Measured denominators kept in profiles/measured_peaks.md (written from
    `bench.py --peaks` and `--copy-calibration`): FP32 VALU lane-slots/s,
    FP32 matrix TFLOP/s, HBM fill GB/s; None when the record is missing or
    the microbenchmarks' source has changed since."""
    path = os.path.join(ROOT, "profiles", "measured_peaks.md")
    try:
        rec = next(json.loads(l.split("record:", 1)[1]) for l in open(path) if l.startswith("record:"))
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                return None
    except (OSError, StopIteration, ValueError, KeyError):
        return None
    return rec


def with_measured_peak(roof, key):
    """Adds the measured peak of the same unit beside the published one."""
    rec = measured_peaks()
    if rec is not None:
        roof["peak_measured"] = rec[key]
        roof["frac_of_measured_peak"] = roof["achieved"] / rec[key]
    return roof


def _timed_steps(step, K, W):
    import torch
    for _ in range(W):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [step() for _ in range(K)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([[a.elapsed_time(b) for a, b in zip(e[:-1], e[1:])] for e in evs])
    return wall, ms.sum(0) / 1e3        # seconds summed over the K steps, per sub-step


B2B_CALLS = 100


def graph_leg(res_fn, eval_fn, work, K, W):
    """The restructure and the redundant evaluation, each recorded once into a
    HIP graph (api.Graph) and replayed: the same kernels on the same arrays,
    without the host launch gaps between them; timed like the steps."""
    from paper_2511_21535_amd import api
    g_res, g_eval = api.Graph(res_fn), api.Graph(eval_fn)

    def step():
        e = _events(3)
        e[0].record()
        g_res.replay()
        e[1].record()
        g_eval.replay()
        e[2].record()
        return e

    _, (t_res, t_red) = _timed_steps(step, K, W)
    return {"ms": {"restructure": t_res / K * 1e3, "eval_redundant": t_red / K * 1e3},
            "rate_incl_restructure": work * K / (t_res + t_red), "rate_excl_restructure": work * K / t_red}


def back_to_back(fns, calls=B2B_CALLS):
    """Mean microseconds per call of each function over `calls` calls issued
    back to back between two events (the queue stays full, so the launch
    gaps of a single timed call are hidden); for the microsecond-scale
    workloads."""
    import torch
    out = {}
    for name, fn in fns.items():
        fn()
        torch.cuda.synchronize()
        ev = _events(2)
        ev[0].record()
        for _ in range(calls):
            fn()
        ev[1].record()
        torch.cuda.synchronize()
        out[name] = ev[0].elapsed_time(ev[1]) * 1e3 / calls
    return out


def _events(k):
    import torch
    return [torch.cuda.Event(enable_timing=True) for _ in range(k)]


def _base(metric, value, unit, K, W, wall, dtype, config, higher=True):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": K, "warmup": W,
            "ms_per_step": wall / K * 1e3, "higher_is_better": higher, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


# --------------------------------------------------------------- CPU oracle
def rel_l2(got, ref):
    """Relative L2 error of `got` against `ref` (both flattened)."""
    got, ref = np.asarray(got).ravel(), np.asarray(ref).ravel()
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def oracle_gravity_sample(x, y, z, m, w, n_leaves_sample, timed=True, min_seconds=10.0, max_reps=8):
    """The FP64 oracle, as it stands, on target leaves of the same workload
    (all of them when n_leaves_sample <= 0, else that many drawn uniformly,
    seed 123).  Returns (baseline, reference): `baseline` is the oracle's
    rate -- pairs evaluated per second of evaluation time, repeated until
    about `min_seconds` have passed (median of the repeats), plus one thread
    on the first 5000 leaves -- or None when not `timed`; `reference` is
    (caller index, phi, ax, ay, az) of the sampled targets.  The oracle's tree
    and brute-force near lists are built first and not timed."""
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
    ref = None
    while len(times) < (max_reps if timed else 1) and (not timed or sum(times) < min_seconds or len(times) < 3):
        t0 = time.perf_counter()
        ref = oracle.gravity_leaves(x, y, z, m, w["eps"], ot, sel, ss, si)
        times.append(time.perf_counter() - t0)
    if not timed:
        return None, ref
    t_eval = float(np.median(times))
    cores = oracle.threads()
    # one thread, on the first leaves of the same selection (about 0.2 s)
    k1 = min(5000, len(sel))
    s1, i1 = ss[:k1 + 1], si[:ss[k1]]
    pairs1 = int((occ[sel[:k1]] * seg[:k1]).sum() - occ[sel[:k1]].sum())
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.gravity_leaves(x, y, z, m, w["eps"], ot, sel[:k1], s1, i1)
        t1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(cores)
    return ({"value": pairs / t_eval, "unit": "pair-interactions/s", "cores": cores,
             "kind": "oracle", **host_cpu(),
             "value_1_thread": pairs1 / t1,
             "sample": f"{what}, {pairs} pairs, FP64 plain loops, median of {len(times)} evaluations "
                       f"of {t_eval:.2f} s (oracle tree build {t_tree:.2f} s and near lists not counted); "
                       f"1 thread: the first {k1} of those leaves, {pairs1} pairs, {t1:.2f} s"}, ref)


def gravity_error(outs, ref):
    """Errors of the GPU results (phi, ax, ay, az: caller-order device
    arrays) against the oracle's on its sampled targets: relative L2 of phi
    and of a (one 3-vector per target), and the largest pointwise error of
    each over the RMS of the oracle's values."""
    idx, phi, ax, ay, az = ref
    idx_t = None
    g = []
    for o in outs:
        if idx_t is None:
            import torch
            idx_t = torch.as_tensor(idx.astype(np.int64), device=o.device)
        g.append(o.index_select(0, idx_t).cpu().numpy())
    a_ref, a_got = np.stack([ax, ay, az]), np.stack(g[1:])
    rms = lambda v: float(np.sqrt(np.mean(np.square(v))))
    return {"phi_rel_l2": rel_l2(g[0], phi), "a_rel_l2": rel_l2(a_got, a_ref),
            "phi_max_abs_over_rms": float(np.max(np.abs(g[0] - phi))) / rms(phi),
            "a_max_abs_over_rms": float(np.max(np.linalg.norm(a_got - a_ref, axis=0))) / rms(np.linalg.norm(a_ref, axis=0)),
            "targets": int(len(idx))}


def host_cpu():
    """The host's processor model and logical CPU count."""
    model = None
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def oracle_helmholtz_sample(sides, q, n_targets, unit, timed=True):
    """The FP64 oracle on `n_targets` targets drawn uniformly (seed 123).
    Returns (baseline, (targets, u)): the oracle's rate on that sample (None
    when not `timed`) and its complex128 results there."""
    import oracle
    n = int(sum(int(s) ** 3 for s in sides))
    rng = np.random.default_rng(123)
    tg = np.sort(rng.choice(n, min(n_targets, n), replace=False)).astype(np.int64)
    sides = np.asarray(sides)
    off = oracle.grid_offsets(sides)
    pairs = 0
    for t in tg:
        g = int(np.searchsorted(off, t, side="right") - 1)
        ns = int(sides[g])
        loc = t - off[g]
        c = np.array([loc % ns, (loc // ns) % ns, loc // (ns * ns)]) // 4
        nb = ns // 4
        pairs += 64 * int(np.prod([min(ci + 1, nb - 1) - max(ci - 1, 0) + 1 for ci in c])) - 1
    t0 = time.perf_counter()
    ref = oracle.helmholtz(sides, q, targets=tg)
    dt = time.perf_counter() - t0
    nrhs = 1 if q.ndim == 1 else q.shape[1]
    if not timed:
        return None, (tg, ref)
    return ({"value": pairs * nrhs / dt, "unit": unit, "cores": oracle.threads(), "kind": "oracle", **host_cpu(),
             "sample": f"{len(tg)} of {n} targets drawn uniformly (seed 123), {pairs} pairs x {nrhs} "
                       f"RHS, complex128, {dt:.2f} s (the time includes the oracle's copy of q to "
                       f"complex128)"}, (tg, ref))


def helmholtz_error(u, ref):
    """Errors of the GPU result u (caller order [n] or [n, R], device) against
    the oracle's on its sampled targets: relative L2 over all sampled values,
    the worst right-hand side's relative L2, and the largest pointwise error
    over the RMS of the oracle's values."""
    import torch
    tg, r = ref
    got = u.index_select(0, torch.as_tensor(tg, device=u.device)).cpu().numpy().astype(np.complex128)
    got, r = got.reshape(len(tg), -1), r.reshape(len(tg), -1)
    per = [rel_l2(got[:, j], r[:, j]) for j in range(r.shape[1])]
    return {"u_rel_l2": rel_l2(got, r), "u_worst_rhs_rel_l2": max(per),
            "u_max_abs_over_rms": float(np.max(np.abs(got - r)) / np.sqrt(np.mean(np.abs(r) ** 2))),
            "targets": int(len(tg)), "rhs": int(r.shape[1])}


# --------------------------------------------------------------- gravity
def run_gravity(wname, args):
    import torch
    from paper_2511_21535_amd import api
    from paper_2511_21535_amd import workloads as W
    dev = torch.device("cuda:0")
    w = W.WORKLOADS[wname]
    x, y, z, m = W.particles(wname)
    gx, gy, gz, gm = (torch.as_tensor(v, device=dev) for v in (x, y, z, m))
    eps, prec = w["eps"], w["prec"]
    mixed = prec == "fp32"
    n = x.shape[0]
    bpe = 16.0 if mixed else 32.0         # bytes per redundant entry

    tree = api.Tree.build_particles(gx, gy, gz, depth=w["depth"], leaf_cap=w["leaf_cap"])
    nbrs = tree.neighbors()
    loc = api.locality(tree, nbrs, bytes_per_entry=bpe, cache_bytes=CACHE_BYTES)
    S, pairs = int(loc["entries"]), int(loc["pairs"])
    red = api.restructure_gravity(tree, nbrs, gx, gy, gz, gm, prec=prec, S=S)
    outs = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4)]

    def step():
        e = _events(6)
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

    K = args.steps
    wall, (t_tree, t_nbr, t_res, t_red, t_gat) = _timed_steps(step, K, args.warmup)
    value = pairs * K / (t_res + t_red)
    rate_red, rate_gat = pairs * K / t_red, pairs * K / t_gat
    slots = SLOTS_PER_PAIR_MIXED if mixed else SLOTS_PER_PAIR_FP64
    achieved = pairs * slots / (t_red / K) / 1e12
    peak = VALU_PEAK_SLOTS / 1e12
    desc = {"gravity_plummer_2m": "2^21 particles, 8 Plummer spheres (scale radii 0.01-0.1), adaptive "
                                  "octree leaf cap 64, eps 1e-3, FP32-mixed",
            "gravity_uniform_4096": "4096 particles uniform in the unit cube, uniform octree depth 3, "
                                    "eps 1e-3, FP64",
            "adjoint_gravity_256k": "2^18 Plummer particles, leaf cap 64, eps 1e-3, FP64"}[wname]
    # algorithmic restructure traffic: segments written once, caller rows read
    # once, sorted rows written and read once
    res_bytes = S * bpe + n * (32 + 2 * 32)
    # algorithmic bytes of the redundant evaluation: the redundant rows read
    # once, four FP64 results written per target, the permutation read once
    eval_bytes = S * bpe + n * (4 * 8 + 4)
    kname = "k_gravity_mixed_red" if mixed else "k_gravity_fp64_red"
    traffic = pmc_traffic(kname, wname, "gravity.hip")
    line = _base(METRIC, value, "pair-interactions/s", K, args.warmup, wall,
                 "f32+f64" if mixed else "f64",
                 {"workload": f"{wname}: {desc}", "n": n, "leaves": tree.n_leaves,
                  "max_level": tree.max_level, "near_entries": nbrs.count, "redundant_entries": S,
                  "pairs": pairs, "parallelism": "single GPU"})
    line.update({
        "rates": {"redundant_incl_restructure": value, "redundant_excl_restructure": rate_red,
                  "gather": rate_gat,
                  "speedup_redundant_vs_gather_incl_restructure": value / rate_gat,
                  "speedup_redundant_vs_gather_kernel_only": rate_red / rate_gat},
        "ms": {"tree": t_tree / K * 1e3, "neighbors": t_nbr / K * 1e3, "restructure": t_res / K * 1e3,
               "eval_redundant": t_red / K * 1e3, "eval_gather": t_gat / K * 1e3},
        "locality": {k: loc[k] for k in ("d_mean", "d_ratio", "v_ratio", "locality")},
        "speedup_model": speedup_model.evaluate({"compute": t_gat}, {"collect": t_res, "compute": t_red},
                                                loc["d_ratio"], loc["v_ratio"], S * bpe, CACHE_BYTES),
        "roofline": with_measured_peak(
            {"bound": "alu", "kernel": kname, "achieved": achieved, "peak": peak,
             "unit": "T VALU lane-slots/s", "frac": achieved / peak,
             "traffic": traffic["bytes"] if traffic else None,
             "traffic_detail": dict(traffic, algorithmic_bytes=eval_bytes) if traffic else None,
             "algorithmic_per_pair": slots}, "valu_T_lane_slots_per_s"),
        "restructure_roofline": with_measured_peak(
            {"bound": "hbm", "achieved": res_bytes / (t_res / K) / 1e9, "peak": 8000.0, "unit": "GB/s",
             "frac": res_bytes / (t_res / K) / 8e12, "bytes": res_bytes}, "hbm_fill_GBps"),
    })
    line["graph"] = graph_leg(
        lambda: api.restructure_gravity(tree, nbrs, gx, gy, gz, gm, prec=prec, out=red),
        lambda: api.gravity(tree, nbrs, eps, layout="redundant", prec=prec, red=red, out=outs), pairs, K, args.warmup)
    if t_red / K < 2e-4:
        b2b = back_to_back({
            "restructure_us": lambda: api.restructure_gravity(tree, nbrs, gx, gy, gz, gm, prec=prec, out=red),
            "eval_redundant_us": lambda: api.gravity(tree, nbrs, eps, layout="redundant", prec=prec, red=red,
                                                     out=outs),
            "eval_gather_us": lambda: api.gravity(tree, nbrs, eps, x=gx, y=gy, z=gz, m=gm, layout="gather",
                                                  prec=prec, out=outs)})
        line["back_to_back"] = dict(b2b, calls=B2B_CALLS)
    # per-interaction layout (records per near-list entry), timed after the
    # steps on the same tree and lists: restructure, then evaluation + update
    inter = api.restructure_interactions(tree, nbrs, gx, gy, gz, gm, prec=prec)

    def step_inter():
        e = _events(3)
        e[0].record()
        api.restructure_interactions(tree, nbrs, gx, gy, gz, gm, prec=prec, out=inter)
        e[1].record()
        api.gravity_interactions(tree, nbrs, inter, eps, out=outs)
        e[2].record()
        return e

    _, (t_ires, t_ieval) = _timed_steps(step_inter, K, args.warmup)
    line["rates"].update({"interaction_incl_restructure": pairs * K / (t_ires + t_ieval),
                          "interaction_excl_restructure": pairs * K / t_ieval})
    line["ms"].update({"interaction_restructure": t_ires / K * 1e3, "interaction_eval": t_ieval / K * 1e3})
    line["interaction_layout"] = {"rows": inter.count, "bytes": inter.count * bpe,
                                  "result_rows": inter.target_rows}
    del inter
    line["periodic"] = periodic_leg(tree, (gx, gy, gz, gm), w, K, args.warmup, bpe,
                                    {"neighbors": t_nbr, "restructure": t_res, "eval_redundant": t_red,
                                     "eval_gather": t_gat})
    line["interaction_types"] = interaction_types_leg((gx, gy, gz, gm), w, K, args.warmup)
    # every result against the FP64 oracle, on the oracle's sample (all leaves
    # when it is timed, 2000 leaves otherwise), for both layouts
    base, ref = oracle_gravity_sample(x, y, z, m, w, args.cpu_leaves if not args.no_cpu else 2000,
                                      timed=not args.no_cpu)
    err = {}
    for layout in ("redundant", "gather"):
        o = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4)]
        api.gravity(tree, nbrs, eps, x=gx, y=gy, z=gz, m=gm, layout=layout, prec=prec, red=red, out=o)
        err[layout] = gravity_error(o, ref)
    line["error_vs_oracle"] = dict(err, precision="FP32-mixed: leaf-relative FP32 positions, FP32 pair terms, "
                                                  "at most 32 summed in FP32, then FP64" if mixed else "FP64")
    if base is not None:
        line["cpu_baseline"] = base
    return line


def interaction_types_leg(src, w, K, W):
    """Local, remote and periodic interactions (Sec. 5.2) of one domain: the
    particles are cut at x = 0.5 into two domains with trees of their own; the
    first domain's targets take local sources (its own tree), remote sources
    (the other domain's points, received in a sharded run) and, on the torus,
    periodic images of both.  Each type is timed as restructure + redundant
    evaluation and as a gather evaluation, the remote type in launches of its
    own (its sums added to the local ones), the periodic images inside the
    local and remote lists.  Eq. (15) gives the local share of the time; Eq.
    (14), read as Eq. (4) on the local part, the speedup had only the local
    part been restructured, beside the measured speedup of restructuring all."""
    import torch
    from paper_2511_21535_amd import api
    eps, prec = w["eps"], w["prec"]
    cut = src[0] < 0.5
    da, db = [v[cut].contiguous() for v in src], [v[~cut].contiguous() for v in src]
    ta = api.Tree.build_particles(*da[:3], depth=w["depth"], leaf_cap=w["leaf_cap"])
    tb = api.Tree.build_particles(*db[:3], depth=w["depth"], leaf_cap=w["leaf_cap"])
    occ = torch.diff(ta.leaf_start).to(torch.int64)
    lists = {"local": ta.neighbors(), "remote": api.build_neighbors(ta, src_tree=tb),
             "local_periodic": ta.neighbors(periodic=True),
             "remote_periodic": api.build_neighbors(ta, periodic=True, src_tree=tb)}
    reds = {k: (api.restructure_remote(ta, tb, nb, *db, prec=prec) if k.startswith("remote")
                else api.restructure_gravity(ta, nb, *da, prec=prec)) for k, nb in lists.items()}
    pairs = {k: int((torch.diff(r.red_start) * occ).sum().item()) - (0 if k.startswith("remote") else ta.n)
             for k, r in reds.items()}
    outs = [torch.empty(ta.n, dtype=torch.float64, device=src[0].device) for _ in range(4)]

    def run(k, layout):
        nb, r = lists[k], reds[k]
        if k.startswith("remote"):
            if layout == "restructure":
                api.restructure_remote(ta, tb, nb, *db, prec=prec, out=r)
            else:
                api.gravity_remote(ta, tb, nb, eps, *da[:3], *db, layout=layout, prec=prec, red=r, out=outs)
        else:
            if layout == "restructure":
                api.restructure_gravity(ta, nb, *da, prec=prec, out=r)
            else:
                api.gravity(ta, nb, eps, *da, layout=layout, prec=prec, red=r, out=outs)

    keys = list(lists)
    seq = [(k, lay) for k in keys for lay in ("restructure", "redundant", "gather")]

    def step():
        e = _events(len(seq) + 1)
        e[0].record()
        for i, (k, lay) in enumerate(seq):
            run(k, lay)
            e[i + 1].record()
        return e

    _, t = _timed_steps(step, K, W)
    ms = {f"{k}_{lay}": t[i] / K * 1e3 for i, (k, lay) in enumerate(seq)}
    red_t = {k: ms[f"{k}_restructure"] + ms[f"{k}_redundant"] for k in keys}
    gat_t = {k: ms[f"{k}_gather"] for k in keys}
    # periodic part: the periodic lists' time beyond the plain lists' (local and remote)
    T = {}
    for name, tt in (("redundant_incl_restructure", red_t), ("gather", gat_t)):
        loc, rem = tt["local"], tt["remote"]
        per = (tt["local_periodic"] - loc) + (tt["remote_periodic"] - rem)
        T[name] = {"local": loc, "remote": rem, "periodic": per,
                   "local_share_eq15": speedup_model.local_share(loc, rem, per)}
    share = T["gather"]["local_share_eq15"]
    x_local = gat_t["local"] / red_t["local"]
    all_gat = gat_t["local_periodic"] + gat_t["remote_periodic"]
    all_red = red_t["local_periodic"] + red_t["remote_periodic"]
    return {
        "domain": "x < 0.5 of the workload (targets); sources: its own points, the other domain's, "
                  "and the periodic images of both",
        "targets": ta.n, "target_leaves": ta.n_leaves, "source_points_remote": tb.n,
        "near_entries": {k: nb.count for k, nb in lists.items()},
        "pairs": pairs,
        "ms": ms,
        "ms_by_type": T,
        "speedup_local_only_eq14": speedup_model.op_speedup(share, x_local),
        "speedup_local_measured": x_local,
        "speedup_all_measured": all_gat / all_red,
        "launches": "local and remote each run in launches of their own (restructure, evaluation); the 26 "
                    "periodic images ride in the local and remote lists",
    }


def periodic_leg(tree, src, w, K, W, bpe, plain):
    """The same tree on the unit torus (periodic images, Sec. 5.2): periodic
    near lists, restructure, redundant and gather evaluations, timed after the
    headline steps.  Eq. (15): the local share of the near-field time is the
    plain (local-only) evaluation time over the periodic one; Eq. (14), read as
    Eq. (4) on the local part, gives the speedup had only the local part been
    restructured, beside the measured speedup of restructuring both."""
    import torch
    from paper_2511_21535_amd import api
    eps, prec = w["eps"], w["prec"]
    nbp = tree.neighbors(periodic=True)
    loc = api.locality(tree, nbp, bytes_per_entry=bpe, cache_bytes=CACHE_BYTES)
    S, pairs = int(loc["entries"]), int(loc["pairs"])
    red = api.restructure_gravity(tree, nbp, *src, prec=prec, S=S)
    outs = [torch.empty(tree.n, dtype=torch.float64, device=src[0].device) for _ in range(4)]

    def step():
        e = _events(5)
        e[0].record()
        nb = tree.neighbors(cap=nbp.count, periodic=True)
        e[1].record()
        r = api.restructure_gravity(tree, nb, *src, prec=prec, out=red)
        e[2].record()
        api.gravity(tree, nb, eps, layout="redundant", prec=prec, red=r, out=outs)
        e[3].record()
        api.gravity(tree, nb, eps, *src, layout="gather", prec=prec, out=outs)
        e[4].record()
        return e

    _, (t_nbr, t_res, t_red, t_gat) = _timed_steps(step, K, W)
    del red
    share = speedup_model.local_share(plain["eval_gather"], 0.0, t_gat - plain["eval_gather"])
    x_local = plain["eval_gather"] / (plain["restructure"] + plain["eval_redundant"])
    return {
        "near_entries": nbp.count, "redundant_entries": S, "pairs": pairs,
        "periodic_entries": int((nbp.nbr_shift != 13).sum().item()),
        "rates": {"redundant_incl_restructure": pairs * K / (t_res + t_red),
                  "redundant_excl_restructure": pairs * K / t_red, "gather": pairs * K / t_gat},
        "ms": {"neighbors": t_nbr / K * 1e3, "restructure": t_res / K * 1e3,
               "eval_redundant": t_red / K * 1e3, "eval_gather": t_gat / K * 1e3},
        "local_share_eq15": share,
        "speedup_local_only_eq14": speedup_model.op_speedup(share, x_local),
        "speedup_both_measured": t_gat / (t_res + t_red),
    }


# --------------------------------------------------------------- Helmholtz
def run_helmholtz(wname, args):
    """Grid workloads.  The redundancy grain (one segment per box, or per tile
    of 2^3 or 4^3 boxes) is picked by timing restructure + redundant
    evaluation at each grain (a leg of its own, reported under "grains"); the
    timed steps then use it.  Evaluations run in FP32_MIXED (each near box's
    FP32 partial product added into FP64 per-target sums); the FP32 mode
    (single precision throughout) is timed beside it, with the error of both
    against the oracle."""
    import torch
    from paper_2511_21535_amd import api, autotune
    from paper_2511_21535_amd import workloads as W
    dev = torch.device("cuda:0")
    w = W.WORKLOADS[wname]
    if wname == "helmholtz_grid_64":
        sides = np.array([w["n_side"]])
    else:
        sides = W.batched_grid_sides(w["n_instances"], w["seed"])
    grids = [api.Grid(int(s), *W.grid_geometry(int(s))) for s in sides]
    nrhs = w["nrhs"]
    prec = "fp32"
    q = W.grid_rhs(int((sides.astype(np.int64) ** 3).sum()), nrhs, seed=w["seed"])
    gq = torch.as_tensor(q if nrhs > 1 else q[:, 0].copy(), device=dev)
    tree = api.Tree.build_grids(grids, device=dev)
    nbrs = tree.neighbors()
    loc = api.locality(tree, nbrs, bytes_per_entry=8.0 * nrhs, cache_bytes=CACHE_BYTES)
    S, pairs = int(loc["entries"]), int(loc["pairs"])
    mfma = nrhs % 32 == 0
    tile, tune_ms = None, {}
    if mfma:
        tile, tune_ms = autotune.tune_helmholtz(tree, nbrs, q=gq, layout="gather", prec=prec)
    out = torch.empty_like(gq)
    K = args.steps
    work = pairs * nrhs
    # the set-up of the evaluation (parameters, G blocks built in FP64, work
    # order), built once per tree like the tree itself; every timed
    # evaluation call then runs only its product (and the gather copy)
    plan = api.HelmholtzPlan(tree, nbrs, prec=prec, nrhs=nrhs, tile=tile)

    # the redundancy grain: restructure + redundant evaluation timed at each grain
    grain_ms = {}
    for g in autotune.GRAINS:
        red = api.restructure(tree, nbrs, [gq], prec=prec, nrhs=nrhs, grain=g)

        def gstep(red=red):
            e = _events(3)
            e[0].record()
            api.restructure(tree, nbrs, [gq], prec=prec, nrhs=nrhs, out=red)
            e[1].record()
            api.helmholtz(tree, nbrs, None, layout="redundant", red=red, out=out, plan=plan)
            e[2].record()
            return e

        _, (t_r, t_e) = _timed_steps(gstep, K, args.warmup)
        grain_ms[g] = {"restructure_ms": t_r / K * 1e3, "eval_redundant_ms": t_e / K * 1e3,
                       "entries": red.count, "bytes": red.count * 8 * nrhs,
                       "rate_incl_restructure": work * K / (t_r + t_e)}
        del red
        torch.cuda.empty_cache()
    grain = min(grain_ms, key=lambda g: grain_ms[g]["restructure_ms"] + grain_ms[g]["eval_redundant_ms"])
    red = api.restructure(tree, nbrs, [gq], prec=prec, nrhs=nrhs, grain=grain)
    S_red = red.count

    def step():
        e = _events(6)
        e[0].record()
        t = api.Tree.build_grids(grids, device=dev)
        e[1].record()
        nb = t.neighbors(cap=nbrs.count)
        e[2].record()
        r = api.restructure(t, nb, [gq], prec=prec, nrhs=nrhs, out=red)
        e[3].record()
        api.helmholtz(t, nb, None, layout="redundant", red=r, out=out, plan=plan)
        e[4].record()
        api.helmholtz(t, nb, gq, layout="gather", out=out, plan=plan)
        e[5].record()
        return e

    wall, (t_tree, t_nbr, t_res, t_red, t_gat) = _timed_steps(step, K, args.warmup)
    value = work * K / (t_res + t_red)
    flops = 8.0 * work
    per_pair = "8 flop per complex multiply-add (x RHS)"
    if mfma:
        kern, src, t_dom = "k_helm_mfma_red", "helmholtz_mfma.hip", t_red / K
        roof = {"bound": "mfma", "peak": FP32_MFMA_PEAK_TFLOPS, "instruction": "v_mfma_f32_32x32x2f32",
                "timed": "the redundant evaluation call from the prepared plan (queue counter reset, product)"}
        # the product form the kernel runs: 64 RHS per wave with the FP64 sums take four
        # real products per complex one, every other multi-RHS shape three (3M)
        if not (tile and tile[2] == 64):
            flops = 6.0 * work
            per_pair = ("6 flop per pair x RHS: the complex multiply-add as three real products "
                        "(Re G Re Q, Im G Im Q, (Re G + Im G)(Re Q + Im Q))")
            roof["achieved_8flop_equivalent"] = 8.0 * work / t_dom / 1e12
        # redundant rows read once, results written once (complex64)
        alg_bytes = S_red * nrhs * 8 + tree.n * nrhs * 8
    elif nrhs == 1:
        # one right-hand side on the matrix cores, target boxes as the columns; the
        # redundant evaluation call from the plan is the product launch alone
        kern, src, t_dom = "k_helm_mfma_cols_red", "helmholtz_cols.hip", t_red / K
        roof = {"bound": "mfma", "peak": FP32_MFMA_PEAK_TFLOPS, "instruction": "v_mfma_f32_16x16x4f32",
                "timed": "the redundant evaluation call from the prepared plan (one product launch)"}
        flops = 6.0 * work
        per_pair = ("6 flop per pair: the complex multiply-add as three real products "
                    "(Re G Re Q, Im G Im Q, (Re G + Im G)(Re Q + Im Q))")
        roof["achieved_8flop_equivalent"] = 8.0 * work / t_dom / 1e12
        # redundant rows read once, results written once (complex64), G blocks read once
        alg_bytes = S_red * 8 + tree.n * 8 + 27 * 4096 * 8
    else:
        kern, src, t_dom = "k_helmholtz_red", "helmholtz.hip", t_red / K
        roof = {"bound": "alu", "peak": FP32_VALU_PEAK_TFLOPS}
        alg_bytes = S_red * nrhs * 8 + tree.n * nrhs * 8
    ach = flops / t_dom / 1e12
    traffic = pmc_traffic(kern, wname, src)
    roof.update({"kernel": kern, "achieved": ach, "unit": "TFLOP/s", "frac": ach / roof["peak"],
                 "traffic": traffic["bytes"] if traffic else None,
                 "traffic_detail": dict(traffic, algorithmic_bytes=alg_bytes) if traffic else None,
                 "algorithmic_per_pair": per_pair})
    unit = "pair-interactions/s" if nrhs == 1 else "pair-RHS-interactions/s"
    desc = ("64^3 grid, leaf boxes of 4^3 points, 1 complex RHS, k at 10 points per wavelength"
            if wname == "helmholtz_grid_64" else
            f"{len(sides)} grids of edge 16..48 (leaf boxes of 4^3 points, k at 10 points per wavelength), "
            f"{nrhs} complex RHS each, one persistent launch on the FP32 matrix cores")
    cfg = {"workload": f"{wname}: {desc}", "grids": len(sides), "points": tree.n, "boxes": tree.n_leaves,
           "nrhs": nrhs, "near_entries": nbrs.count, "redundant_entries": S_red, "box_grain_entries": S,
           "grain": grain, "pairs": pairs, "precision": "FP32_MIXED",
           "tile": list(tile) if tile else None, "parallelism": "single GPU"}
    line = _base(METRIC + ("" if nrhs == 1 else ", x RHS"), value, unit, K, args.warmup, wall,
                 "f32 (complex64) + f64 sums", cfg)
    line.update({
        "rates": {"redundant_incl_restructure": value, "redundant_excl_restructure": work * K / t_red,
                  "gather": work * K / t_gat,
                  "speedup_redundant_vs_gather_incl_restructure": t_gat / (t_res + t_red),
                  "speedup_redundant_vs_gather_kernel_only": t_gat / t_red},
        "ms": {"tree": t_tree / K * 1e3, "neighbors": t_nbr / K * 1e3, "restructure": t_res / K * 1e3,
               "eval_redundant": t_red / K * 1e3, "eval_gather": t_gat / K * 1e3},
        "grains": {str(g): dict(v, speedup_vs_gather_incl_restructure=(t_gat / K * 1e3) /
                                (v["restructure_ms"] + v["eval_redundant_ms"]))
                   for g, v in grain_ms.items()},
        "locality": {k: loc[k] for k in ("d_mean", "d_ratio", "v_ratio", "locality")},
        "speedup_model": speedup_model.evaluate({"compute": t_gat}, {"collect": t_res, "compute": t_red},
                                                loc["d_ratio"], loc["v_ratio"], S * 8.0 * nrhs, CACHE_BYTES),
        "roofline": with_measured_peak(roof, "mfma_f32_TFLOPs") if roof["bound"] == "mfma" else roof,
    })
    line["locality"]["note"] = "box grain (V = S x 8 x RHS bytes), as Definition 1 states it"
    # FP32 throughout: the same layouts and kernels without the FP64 sums
    plain_tile = None
    if mfma:
        plain_tile, _ = autotune.tune_helmholtz(tree, nbrs, q=gq, layout="gather", prec="fp32_plain")
    plain_plan = api.HelmholtzPlan(tree, nbrs, prec="fp32_plain", nrhs=nrhs, tile=plain_tile)

    def pstep():
        e = _events(3)
        e[0].record()
        api.helmholtz(tree, nbrs, None, layout="redundant", red=red, out=out, plan=plain_plan)
        e[1].record()
        api.helmholtz(tree, nbrs, gq, layout="gather", out=out, plan=plain_plan)
        e[2].record()
        return e

    _, (tp_red, tp_gat) = _timed_steps(pstep, K, args.warmup)
    line["fp32_plain"] = {"ms": {"eval_redundant": tp_red / K * 1e3, "eval_gather": tp_gat / K * 1e3},
                          "tile": list(plain_tile) if plain_tile else None,
                          "cost_of_fp64_sums": {"redundant": t_red / tp_red, "gather": t_gat / tp_gat}}
    if t_red / K < 2e-4:
        b2b = back_to_back({
            "restructure_us": lambda: api.restructure(tree, nbrs, [gq], prec=prec, nrhs=nrhs, out=red),
            "eval_redundant_us": lambda: api.helmholtz(tree, nbrs, None, layout="redundant", red=red, out=out,
                                                       plan=plan),
            "eval_gather_us": lambda: api.helmholtz(tree, nbrs, gq, layout="gather", out=out, plan=plan)})
        line["back_to_back"] = dict(b2b, calls=B2B_CALLS)
        if kern == "k_helm_mfma_cols_red":
            # a launch of tens of microseconds: its average duration is taken over
            # B2B_CALLS launches issued back to back between two HIP events on the
            # library's stream (a single timed call also holds the host's launch gap)
            rl = line["roofline"]
            rl["achieved_single_call"] = rl["achieved"]
            rl["achieved"] = flops / (b2b["eval_redundant_us"] * 1e-6) / 1e12
            rl["achieved_8flop_equivalent"] = 8.0 * work / (b2b["eval_redundant_us"] * 1e-6) / 1e12
            rl["frac"] = rl["achieved"] / rl["peak"]
            if "peak_measured" in rl:
                rl["frac_of_measured_peak"] = rl["achieved"] / rl["peak_measured"]
            rl["timed"] = (f"the redundant evaluation call from the prepared plan (one product launch), mean of "
                           f"{B2B_CALLS} launches back to back")
    if tile:
        # the best launch shape with 1, 2, 4 and 8 copies of the G blocks (ms per call)
        line["g_block_copies_ms"] = {json.loads(k)[3]: v for k, v in tune_ms.items()
                                     if json.loads(k)[:3] == list(tile[:3])}
    # every result against the FP64 oracle on sampled targets, both layouts, both modes
    n_tg = (20000 if nrhs == 1 else 3000) if not args.no_cpu else (2000 if nrhs == 1 else 200)
    base, ref = oracle_helmholtz_sample(sides, q if nrhs > 1 else q[:, 0], n_tg, unit, timed=not args.no_cpu)
    del q
    err = {}
    for p_, t_ in (("fp32_mixed", (prec, tile)), ("fp32_plain", ("fp32_plain", plain_tile))):
        for layout in ("redundant", "gather"):
            o = torch.empty_like(gq)
            api.helmholtz(tree, nbrs, gq if layout == "gather" else None, layout=layout, prec=t_[0], red=red,
                          nrhs=nrhs, tile=t_[1], out=o)
            err[f"{p_}_{layout}"] = helmholtz_error(o, ref)
            del o
    form = ("three real products" if not (tile and tile[2] == 64) else "four real products")
    line["error_vs_oracle"] = dict(
        err, precision=f"fp32_mixed: FP32 matrix cores (complex as {form}), each near box's 64-term "
                       "partial product added into FP64 sums per target; fp32_plain: all 27 boxes summed in FP32")
    if base is not None:
        line["cpu_baseline"] = base
    return line


# --------------------------------------------------------------- adjoint
def run_adjoint(wname, args):
    import torch
    from paper_2511_21535_amd import api
    from paper_2511_21535_amd import workloads as W
    dev = torch.device("cuda:0")
    w = W.WORKLOADS[wname]
    if w["kind"] == "helmholtz":
        return run_adjoint_helmholtz(wname, args)
    x, y, z, m = W.particles(wname)
    n = len(x)
    g = [torch.as_tensor(W.normal_like(n, seed=w["seed"] + 10 * k), device=dev) for k in range(1, 5)]
    gx, gy, gz, gm = (torch.as_tensor(v, device=dev) for v in (x, y, z, m))
    tree = api.Tree.build_particles(gx, gy, gz, depth=w["depth"], leaf_cap=w["leaf_cap"])
    nbrs = tree.neighbors()
    pairs = int(api.locality(tree, nbrs)["pairs"])

    def step():
        e = _events(4)
        e[0].record()
        api.gravity(tree, nbrs, w["eps"], x=gx, y=gy, z=gz, m=gm, prec="fp64")
        e[1].record()
        api.gravity_adjoint(tree, nbrs, w["eps"], gx, gy, gz, gm, *g)
        e[2].record()
        api.gravity_adjoint(tree, nbrs, w["eps"], gx, gy, gz, gm, *g, prec="fp32")
        e[3].record()
        return e

    K = args.steps
    wall, (t_fwd, t_adj, t_adj32) = _timed_steps(step, K, args.warmup)
    value = pairs * K / (t_fwd + t_adj)
    line = _base("near-field pair-interactions/s, forward + adjoint (gather, FP64)", value,
                 "pair-interactions/s", K, args.warmup, wall, "f64",
                 {"workload": f"{wname}: 2^18 particles, 8 Plummer spheres, adaptive octree leaf cap 64, eps 1e-3; "
                              "forward and adjoint (gradients w.r.t. masses and positions)",
                  "n": n, "leaves": tree.n_leaves, "pairs": pairs, "parallelism": "single GPU"})
    line["ms"] = {"forward": t_fwd / K * 1e3, "adjoint": t_adj / K * 1e3, "adjoint_fp32_mixed": t_adj32 / K * 1e3}
    line["rates"] = {"forward_plus_adjoint": value, "adjoint": pairs * K / t_adj,
                     "adjoint_fp32_mixed": pairs * K / t_adj32}
    peak = VALU_PEAK_SLOTS / 1e12
    ach = pairs * SLOTS_PER_PAIR_ADJ_FP64 / (t_adj / K) / 1e12
    ach32 = pairs * SLOTS_PER_PAIR_ADJ_MIXED / (t_adj32 / K) / 1e12
    traffic = pmc_traffic("k_gravity_adjoint_fp64", wname, "gravity.hip")
    line["roofline"] = with_measured_peak(
        {"bound": "alu", "kernel": "k_gravity_adjoint<FP64>", "achieved": ach, "peak": peak,
         "unit": "T VALU lane-slots/s", "frac": ach / peak,
         "traffic": traffic["bytes"] if traffic else None,
         "algorithmic_per_pair": SLOTS_PER_PAIR_ADJ_FP64}, "valu_T_lane_slots_per_s")
    line["roofline_fp32_mixed"] = with_measured_peak(
        {"bound": "alu", "kernel": "k_gravity_adjoint<FP32_MIXED>", "achieved": ach32, "peak": peak,
         "unit": "T VALU lane-slots/s", "frac": ach32 / peak,
         "algorithmic_per_pair": SLOTS_PER_PAIR_ADJ_MIXED}, "valu_T_lane_slots_per_s")
    # gradients against the oracle's reverse-mode derivative on sampled leaves
    import oracle
    ot = oracle.build_tree_particles(x, y, z, depth=w["depth"], leaf_cap=w["leaf_cap"])
    k = min(2000 if args.no_cpu else 6000, ot.n_leaves)
    sel = np.sort(np.random.default_rng(123).choice(ot.n_leaves, k, replace=False)).astype(np.int32)
    ss, si = oracle.neighbors(ot, sel)
    occ = np.diff(ot.leaf_start).astype(np.int64)
    spairs = int((occ[sel] * np.add.reduceat(occ[si], ss[:-1])).sum() - occ[sel].sum())
    gh = [v.cpu().numpy() for v in g]
    t0 = time.perf_counter()
    idx, rm, rx, ry, rz = oracle.gravity_adjoint_leaves(x, y, z, m, w["eps"], *gh, ot, sel, ss, si)
    dt = time.perf_counter() - t0
    it = torch.as_tensor(idx.astype(np.int64), device=dev)
    err = {}
    for name, prec in (("fp64", "fp64"), ("fp32_mixed", "fp32")):
        gx_, gy_, gz_, gm_ = (v.index_select(0, it).cpu().numpy()
                              for v in api.gravity_adjoint(tree, nbrs, w["eps"], gx, gy, gz, gm, *g, prec=prec))
        err[name] = {"grad_m_rel_l2": rel_l2(gm_, rm),
                     "grad_x_rel_l2": rel_l2(np.stack([gx_, gy_, gz_]), np.stack([rx, ry, rz]))}
    line["error_vs_oracle"] = dict(err, targets=int(len(idx)))
    if not args.no_cpu:
        line["cpu_baseline"] = {"value": spairs / dt, "unit": "pair-interactions/s", "cores": oracle.threads(),
                                "kind": "oracle", **host_cpu(),
                                "sample": f"adjoint only: {k} of {ot.n_leaves} target leaves drawn uniformly "
                                          f"(seed 123), {spairs} pairs, FP64 reverse-mode pair terms, {dt:.2f} s"}
    return line


def run_adjoint_helmholtz(wname, args):
    """Forward and adjoint (A^T g, the transpose action; A is symmetric by
    reciprocity) of the grid operator, FP64 gather, one right-hand side."""
    import torch
    from paper_2511_21535_amd import api
    from paper_2511_21535_amd import workloads as W
    dev = torch.device("cuda:0")
    w = W.WORKLOADS[wname]
    n_side = w["n_side"]
    grids = [api.Grid(n_side, *W.grid_geometry(n_side))]
    tree = api.Tree.build_grids(grids, device=dev)
    nbrs = tree.neighbors()
    pairs = int(api.locality(tree, nbrs)["pairs"])
    q = torch.as_tensor(W.grid_rhs(tree.n, 1, seed=w["seed"])[:, 0].astype(np.complex128), device=dev)
    g = torch.as_tensor(W.grid_rhs(tree.n, 1, seed=w["seed"] + 10)[:, 0].astype(np.complex128), device=dev)

    g32 = g.to(torch.complex64)

    def step():
        e = _events(4)
        e[0].record()
        api.helmholtz(tree, nbrs, q, prec="fp64")
        e[1].record()
        api.helmholtz_adjoint(tree, nbrs, g, prec="fp64")
        e[2].record()
        api.helmholtz_adjoint(tree, nbrs, g32, prec="fp32")
        e[3].record()
        return e

    K = args.steps
    wall, (t_fwd, t_adj, t_adj32) = _timed_steps(step, K, args.warmup)
    value = pairs * K / (t_fwd + t_adj)
    line = _base("near-field pair-interactions/s, forward + adjoint (gather, FP64)", value,
                 "pair-interactions/s", K, args.warmup, wall, "f64 (complex128)",
                 {"workload": f"{wname}: 48^3 grid, 1 RHS, k at 10 points per wavelength; forward and adjoint "
                              "(A^T g, the gradient w.r.t. complex source strengths)",
                  "n": tree.n, "boxes": tree.n_leaves, "pairs": pairs, "parallelism": "single GPU"})
    line["ms"] = {"forward": t_fwd / K * 1e3, "adjoint": t_adj / K * 1e3, "adjoint_fp32": t_adj32 / K * 1e3}
    line["rates"] = {"forward_plus_adjoint": value, "adjoint": pairs * K / t_adj, "adjoint_fp32": pairs * K / t_adj32}
    # both adjoints (A^T g = A g, A symmetric: the forward product on g) on the
    # matrix cores with the target boxes as the columns, the complex multiply-add
    # of a pair as three real products (6 flop executed; the 8-flop equivalent of
    # the four-product form beside it): FP64 on the FP64 matrix instructions, FP32
    # on the FP32 ones (a tile's offsets shared by two workgroups on this grid)
    a64 = 6.0 * pairs / (t_adj / K) / 1e12
    a32 = 6.0 * pairs / (t_adj32 / K) / 1e12
    per_pair = ("6 flop per pair: the complex multiply-add as three real products "
                "(Re G Re Q, Im G Im Q, (Re G + Im G)(Re Q + Im Q))")
    line["roofline"] = {"bound": "mfma", "kernel": "k_helm_mfma_cols64", "achieved": a64,
                        "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": a64 / FP64_MFMA_PEAK_TFLOPS,
                        "traffic": None, "algorithmic_per_pair": per_pair,
                        "achieved_8flop_equivalent": a64 * 8.0 / 6.0,
                        "timed": "the whole adjoint call (sorted copy, G blocks, cleared output, product)"}
    line["roofline_fp32"] = with_measured_peak(
        {"bound": "mfma", "kernel": "k_helm_mfma_cols", "achieved": a32, "peak": FP32_MFMA_PEAK_TFLOPS,
         "unit": "TFLOP/s", "frac": a32 / FP32_MFMA_PEAK_TFLOPS, "algorithmic_per_pair": per_pair,
         "achieved_8flop_equivalent": a32 * 8.0 / 6.0,
         "timed": "the whole adjoint call (sorted copy, G blocks, product)"}, "mfma_f32_TFLOPs")
    # A^T g against the oracle's transpose action (a scatter over every target's near field)
    import oracle
    gh = g.cpu().numpy()
    t0 = time.perf_counter()
    ref = oracle.helmholtz_transpose([n_side], gh)
    dt = time.perf_counter() - t0
    err = {}
    for name, gg, prec in (("fp64", g, "fp64"), ("fp32", g32, "fp32")):
        got = api.helmholtz_adjoint(tree, nbrs, gg, prec=prec).cpu().numpy().astype(np.complex128)
        err[name] = {"grad_rel_l2": rel_l2(got, ref)}
    line["error_vs_oracle"] = dict(err, targets=int(tree.n))
    if not args.no_cpu:
        line["cpu_baseline"] = {"value": pairs / dt, "unit": "pair-interactions/s", "cores": oracle.threads(),
                                "kind": "oracle", **host_cpu(),
                                "sample": f"the whole adjoint (A^T g by scattering every target's near field), "
                                          f"{pairs} pairs, complex128, {dt:.2f} s"}
    return line


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the near-field path is built and measured for a single MI355X.", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.peaks:
        peaks()
        return
    wl = args.workload
    line = run_workload(wl, args)
    if wl == DEFAULT_WORKLOAD and not args.no_nested:
        # the largest gravity configuration, measured the same way, nested in the line
        sub = run_workload(NESTED_WORKLOAD, args)
        line[NESTED_WORKLOAD] = {k: v for k, v in sub.items()
                                 if k not in ("n_gpus", "steps", "warmup", "higher_is_better", "scaling",
                                              "vs_baseline", "data")}
    print(json.dumps(line), flush=True)


def run_workload(wl, args):
    import torch
    torch.cuda.synchronize()
    if wl.startswith("helmholtz"):
        line = run_helmholtz(wl, args)
    elif wl.startswith("adjoint"):
        line = run_adjoint(wl, args)
    else:
        line = run_gravity(wl, args)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return line


if __name__ == "__main__":
    main()

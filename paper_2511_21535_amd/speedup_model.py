"""The paper's analytical speedup model (Sec. 3.2-3.4), fed with measured
component times and the Locality metric.

The model composes the speedup of a restructured operator from the speedups
of its components, each weighted by its share of the baseline time:

  Eq. (4)/(5): X = 1 / (share / X_op + (1 - share))       one restructured part
  Eq. (6):     X_p2p = 1 / sum_c share_c / X_c             collect, transfer,
                                                            compute, update
  Eq. (7):     X_mem-op ~ X_complexity * X_volume           collect and update
  Eq. (8):     X_transfer ~ V_base / V_restructured
  Eq. (9):     X_compute = X_complexity * X_locality * X_launch
  Eq. (10):    X_locality ~ D' V'   if the restructured volume fits the cache
  Eq. (11):    X_locality ~ V' / D' otherwise
  Eq. (15):    share_local = T_local / (T_local + T_remote + T_periodic)

Readings (the paper states proportionalities, not constants): every "~" is
taken with constant 1; Eq. (14) is read as Eq. (4) applied to the local part
(its printed form lacks the reciprocal); a component that only the
restructured version has (the restructure itself, when the baseline collects
nothing) enters Eq. (6) through its time ratio share_c / X_c = t_c,rest /
T_base, the limit of that term.  Host arithmetic only.
"""
from __future__ import annotations

from typing import Dict


def op_speedup(share: float, x_op: float) -> float:
    """Eq. (4)/(5): speedup of the whole when a part with baseline share
    `share` runs x_op times faster."""
    return 1.0 / (share / x_op + (1.0 - share))


def p2p_speedup(t_base: Dict[str, float], t_rest: Dict[str, float]) -> float:
    """Eq. (6) from component times: sum_c share_c / X_c with share_c =
    t_c,base / T_base and X_c = t_c,base / t_c,rest, i.e. sum_c t_c,rest /
    T_base (which also covers a component absent from the baseline)."""
    total = sum(t_base.values())
    return 1.0 / sum(t_rest.get(c, 0.0) / total for c in set(t_base) | set(t_rest))


def locality_factor(d_ratio: float, v_ratio: float, v_rest: float, cache: float) -> float:
    """Eq. (10)/(11): D'V' if the restructured data fits the cache, else V'/D'."""
    return d_ratio * v_ratio if v_rest <= cache else v_ratio / d_ratio


def compute_speedup(x_complexity: float, x_locality: float, x_launch: float = 1.0) -> float:
    """Eq. (9)."""
    return x_complexity * x_locality * x_launch


def memory_op_speedup(x_complexity: float, x_volume: float) -> float:
    """Eq. (7), collect and update."""
    return x_complexity * x_volume


def transfer_speedup(v_base: float, v_rest: float) -> float:
    """Eq. (8)."""
    return v_base / v_rest


def local_share(t_local: float, t_remote: float = 0.0, t_periodic: float = 0.0) -> float:
    """Eq. (15)."""
    return t_local / (t_local + t_remote + t_periodic)


def evaluate(t_base: Dict[str, float], t_rest: Dict[str, float], d_ratio: float, v_ratio: float,
             v_rest: float, cache: float, x_complexity_kernel: float = 1.0, x_launch: float = 1.0) -> dict:
    """Measured versus modelled speedup of the restructured operator.

    t_base / t_rest: component times (keys among collect, transfer, compute,
    update; missing = 0).  The model predicts the compute speedup from Eq.
    (9)-(11); the other components keep their measured times, so the
    predicted total isolates the kernel model."""
    measured_total = p2p_speedup(t_base, t_rest)
    x_compute_measured = t_base["compute"] / t_rest["compute"]
    x_loc = locality_factor(d_ratio, v_ratio, v_rest, cache)
    x_compute_model = compute_speedup(x_complexity_kernel, x_loc, x_launch)
    t_rest_model = dict(t_rest, compute=t_base["compute"] / x_compute_model)
    total = sum(t_base.values())
    return {
        "shares_base": {c: t / total for c, t in t_base.items()},
        "x_compute_measured": x_compute_measured,
        "x_locality_model": x_loc,
        "x_compute_model": x_compute_model,
        "x_p2p_measured": measured_total,
        "x_p2p_model": p2p_speedup(t_base, t_rest_model),
        "formula": "(10) D'V'" if v_rest <= cache else "(11) V'/D'",
    }

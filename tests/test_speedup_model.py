"""The paper's speedup model (Sec. 3.2-3.4), host arithmetic: special cases
and invariants that any correct composition satisfies."""
import math

import pytest

from paper_2511_21535_amd import speedup_model as M


def test_op_speedup_limits():
    assert M.op_speedup(0.0, 7.0) == 1.0            # an untouched part changes nothing
    assert M.op_speedup(0.4, 1.0) == 1.0            # no speedup of the part, none overall
    assert M.op_speedup(1.0, 3.0) == pytest.approx(3.0)
    # Amdahl: the whole is bounded by 1 / (1 - share)
    assert M.op_speedup(0.75, 1e12) == pytest.approx(4.0, rel=1e-9)
    assert M.op_speedup(0.5, 2.0) < M.op_speedup(0.5, 4.0) < 2.0


def test_p2p_speedup_is_the_time_ratio():
    base = {"collect": 1.0, "transfer": 2.0, "compute": 5.0, "update": 2.0}
    rest = {"collect": 3.0, "transfer": 2.5, "compute": 1.0, "update": 1.5}
    assert M.p2p_speedup(base, rest) == pytest.approx(sum(base.values()) / sum(rest.values()))
    # one changed component: Eq. (6) reduces to Eq. (4)
    rest1 = dict(base, compute=2.5)
    assert M.p2p_speedup(base, rest1) == pytest.approx(M.op_speedup(0.5, 2.0))
    # a component only the restructured version has adds its time
    assert M.p2p_speedup({"compute": 4.0}, {"collect": 1.0, "compute": 2.0}) == pytest.approx(4.0 / 3.0)


def test_locality_branches():
    assert M.locality_factor(1.0, 1.0, 10.0, 5.0) == 1.0       # nothing restructured
    assert M.locality_factor(4.0, 0.5, 1.0, 2.0) == 2.0        # fits: D'V'
    assert M.locality_factor(4.0, 0.5, 3.0, 2.0) == 0.125      # exceeds: V'/D'
    assert M.compute_speedup(2.0, 0.5, 3.0) == 3.0
    assert M.memory_op_speedup(0.5, 4.0) == 2.0
    assert M.transfer_speedup(8.0, 2.0) == 4.0
    assert M.local_share(3.0, 1.0, 0.0) == 0.75


def test_evaluate_consistency():
    base = {"compute": 6.0}
    rest = {"collect": 1.0, "compute": 3.0}
    r = M.evaluate(base, rest, d_ratio=4.0, v_ratio=0.5, v_rest=1.0, cache=2.0)
    assert r["x_compute_measured"] == 2.0 and r["x_compute_model"] == 2.0 and r["formula"].startswith("(10)")
    # a model locality equal to the measured kernel speedup reproduces the measurement
    assert r["x_p2p_model"] == pytest.approx(r["x_p2p_measured"]) == pytest.approx(1.5)
    r2 = M.evaluate(base, rest, d_ratio=4.0, v_ratio=0.5, v_rest=3.0, cache=2.0)
    assert r2["x_compute_model"] == 0.125 and math.isclose(r2["x_p2p_model"], 6.0 / (1.0 + 48.0))

"""Host logic of bench.py's instruction-mix ceiling: with given issue rates and the committed
counts per node interaction it is the closed form of the model, and it is absent without the
rates or with counters of another kernel source."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_ceiling_closed_form():
    f = bench.profile_value(bench.VALU_FILE, "far_fp64_f64_lane_instructions_per_node_interaction")
    tr = bench.profile_value(bench.VALU_FILE, "far_fp64_trans_per_node_interaction")
    if f is None or tr is None:
        pytest.skip("the committed counters are from another kernel source")
    rates = {"fma_f64": 5.0e11, "rsq_f64": 1.5e11, "f64_one_rsq_in_nine": 4.5e11,
             "fma_f32": 5.5e11, "rsq_f32": 3.0e11, "f32_one_rsq_in_nine": 5.4e11}
    c = bench.issue_ceiling(rates, "far_fp64", 5.75e12, 2900.0)
    t_rsq = 9.0 / 4.5e11 - 8.0 / 5.0e11          # one reciprocal square root in an FMA stream
    t = (f - tr) / 5.0e11 + tr * t_rsq            # per wavefront of 64 node interactions
    assert c["node_interactions_per_s"] == pytest.approx(64.0 / t, rel=1e-12)
    assert c["achieved_node_interactions_per_s"] == pytest.approx(5.75e12 / 2.9, rel=1e-12)
    assert c["frac"] == pytest.approx(5.75e12 / 2.9 * t / 64.0, rel=1e-12)
    # a quarter-rate reciprocal square root that the FMAs do not hide costs four FMA slots
    slow = dict(rates, f64_one_rsq_in_nine=9.0 / (8.0 / 5.0e11 + 4.0 / 5.0e11))
    c4 = bench.issue_ceiling(slow, "far_fp64", 5.75e12, 2900.0)
    assert c4["node_interactions_per_s"] == pytest.approx(64.0 * 5.0e11 / (f - tr + 4.0 * tr), rel=1e-12)


def test_ceiling_absent_without_rates_or_counters():
    assert bench.issue_ceiling(None, "far_fp64", 5.75e12, 2900.0) is None
    rates = {"fma_f64": 5.0e11, "f64_one_rsq_in_nine": 4.5e11}
    assert bench.issue_ceiling(rates, "no_such_kernel", 5.75e12, 2900.0) is None

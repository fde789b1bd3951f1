"""Host logic of bench.py: the roofline object of every workload (with and
without a beam count in its totals), and measured HBM traffic reported only
for the profiled workload, beam set and kernel source."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def prof(sum_ms, int_ms, n=16):
    return {"sum_points": (n, sum_ms), "integrate": (n, int_ms)}


@pytest.mark.parametrize("kind", ["grid", "homogeneous", "layered"])
def test_roofline_without_a_beam_count(kind):
    roof, name = bench.roofline({"beam_steps": 1e9, "ev_rec": 1e10}, prof(100.0, 50.0), kind)
    assert name == "sum_points"
    assert roof["traffic"] is None
    assert roof["achieved"] == pytest.approx(1e10 * bench.FLOP_POINT_EVAL / 0.1 / 1e12)
    assert roof["frac"] == pytest.approx(roof["achieved"] * 1e12 / bench.PEAK_FP64)


def test_traffic_only_for_the_profiled_beam_set():
    t = bench.TRAFFIC["sum_points"]
    tot = {"beam_steps": 1e9, "ev_rec": 1e10, "beams": t["beams"]}
    roof, _ = bench.roofline(tot, prof(100.0, 50.0), "grid", default_workload=True)
    assert roof["traffic"] == t["bytes_per_launch"]
    tot["beams"] = t["beams"] + 1
    roof, _ = bench.roofline(tot, prof(100.0, 50.0), "grid", default_workload=True)
    assert roof["traffic"] is None
    tot["beams"] = t["beams"]
    roof, _ = bench.roofline(tot, prof(100.0, 50.0), "grid", default_workload=False)
    assert roof["traffic"] is None


def test_dominant_kernel_is_the_longer_one():
    roof, name = bench.roofline({"beam_steps": 1e9, "ev_rec": 1e10, "beams": 5}, prof(10.0, 50.0), "grid")
    assert name == "integrate"
    assert roof["flop_per_unit"] == bench.FLOP_BEAM_STEP["grid"]

"""Host-side pieces of bench.py: the roofline objects of the bench line and
the keying of the stored HBM traffic counters.  No device work."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

N256 = 256 ** 3
# class -> (total ms, launches) as the box's event timing reports it
TIMING = {"nonadv_face": (21.15, 30), "nonadv_update": (4.04, 10), "adv_face": (9.8, 20), "tail": (0.38, 1)}


def test_dominant_class_and_its_figures():
    r = bench._roofline(TIMING, N256, 8, "c2")
    assert r["kernel"] == "nonadv_face" and r["launches"] == 30
    assert r["avg_launch_ms"] == pytest.approx(0.705, abs=1e-4)
    # algorithmic bytes: values per cell x 8 B x cells; flops per face x cells
    assert r["alg_bytes_per_launch"] == round(bench.ALG_VALUES["nonadv_face"] * 8 * N256)
    assert r["alg_flops_per_launch"] == round(bench.ALG_FLOPS["nonadv_face"] * N256)
    tf = bench.ALG_FLOPS["nonadv_face"] * N256 / 0.705e-3 / 1e12
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == 78.6
    assert r["achieved"] == pytest.approx(tf, abs=0.01)
    assert r["frac"] == pytest.approx(tf / 78.6, abs=1e-4)
    # FP32 state: half the bytes, the FP32 vector peak
    r32 = bench._roofline(TIMING, N256, 4, "c3")
    assert abs(r32["alg_bytes_per_launch"] * 2 - r["alg_bytes_per_launch"]) <= 1 and r32["peak"] == 157.3


def test_face_flop_count_is_the_documented_sum():
    # per variable: slope 11, interface 5, Steps 2-5 70 (six variables); the
    # face solve 385; the x launch adds 57 for the m, E, e update
    assert bench.FACE_FLOPS == 901
    assert bench.ALG_FLOPS["nonadv_face"] == pytest.approx((3 * 901 + 57) / 3)


def test_traffic_reported_only_for_its_workload_and_sources():
    key = ("c2", 8, "nonadv_face")
    assert key in bench.TRAFFIC
    h, nbytes = bench.TRAFFIC[key]
    r = bench._roofline(TIMING, N256, 8, "c2")
    assert r["traffic"] == (nbytes if h == bench._kernel_source_hash() else None)
    # other workloads, options that change the face kernels, other precisions
    for wl, esz in (("c2+gravity", 8), ("c2+ionisation", 8), ("c2", 4), ("c3", 4), ("c4", 4)):
        assert bench._roofline(TIMING, N256, esz, wl)["traffic"] is None, wl


def test_traffic_is_dropped_once_the_sources_change(monkeypatch):
    h, nbytes = bench.TRAFFIC[("c2", 8, "nonadv_face")]
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: h)
    assert bench._roofline(TIMING, N256, 8, "c2")["traffic"] == nbytes
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda: "0" * 16)
    assert bench._roofline(TIMING, N256, 8, "c2")["traffic"] is None


def test_step_roofline():
    s = bench._step_roofline(1.0e9, 8)
    assert s["alg_bytes_per_cell_update"] == 126 * 8
    assert s["achieved_gbs"] == pytest.approx(1008.0)
    assert s["frac"] == pytest.approx(1008.0 / 8000.0, abs=1e-4)
    assert bench._step_roofline(1.0e9, 4)["alg_bytes_per_cell_update"] == 504

"""The cost model of Sect. 3.2.2 reproduces the paper's printed numbers."""
import json
import os

import pytest

from paper_2604_11008_amd import accounting

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_cpu_delegated_model_reproduces_the_printed_table():
    g = json.load(open(os.path.join(GOLDEN, "cpu_delegated_model.json")))
    pr = g["printed"]
    m = accounting.cpu_delegated_model(g["float64_arrays_per_particle"], g["bytes_per_value"],
                                       g["particles_per_rank"], g["pcie_one_way_GBps"],
                                       g["single_core_triad_GBps"])
    assert round(m["volume_GB"], 1) == pr["volume_GB"]
    assert abs(m["d2h_ms"] - pr["d2h_ms"]) < 1.0
    assert abs(m["h2d_ms"] - pr["h2d_ms"]) < 1.0
    assert abs(m["pack_ms"] - pr["pack_ms"]) < 1.0
    assert abs(m["unpack_ms"] - pr["unpack_ms"]) < 1.0
    # the paper adds its rounded phases: 2 x (113 + 176) = 578
    assert 2 * (round(m["d2h_ms"]) + round(m["pack_ms"])) == pr["cpu_delegated_total_ms"]
    assert m["total_ms"] == pytest.approx(pr["cpu_delegated_total_ms"], rel=0.005)
    assert pr["gpu_pack_ms"] + pr["gpu_unpack_ms"] == pr["gpu_total_ms"]
    assert round(pr["cpu_delegated_total_ms"] / pr["gpu_total_ms"], 1) == pr["speedup"]
    share = 2 * pr["cpu_delegated_total_ms"] / pr["step_ms"]
    assert round(share, 2) == pr["share_cpu_delegated"]
    # the paper divides its rounded share: 0.78 / 8.0 = 0.0975
    assert round(round(share, 2) / pr["speedup"], 4) == pytest.approx(pr["share_gpu_native"], abs=5.01e-4)


def test_record_sizes():
    assert accounting.record_bytes("f64") == 64
    assert accounting.record_bytes("mixed") == 48
    b = accounting.step_algorithmic_bytes(1000, 10, 500, "f64")
    assert b["step"] == 1000 * 128 + 500 * 24 + 10 * 128


def test_mid_step_record_is_the_papers_17_arrays():
    # Sect. 3.2.2: positions and velocities of both RK2 stages, dV/dt, id and
    # diameter: (2 + 2 + 1) x 3 + 2 = 17 Float64 values per particle
    assert accounting.mid_record_bytes("f64") == 17 * 8
    b = accounting.staged_algorithmic_bytes(10, 2, 1, 5, "f64")
    assert b["stage_kernels"] == 10 * 2 * (64 + 136) + 5 * 24
    assert b["exchange"] == 2 * 2 * 136 + 1 * 2 * 64

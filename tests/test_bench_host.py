"""Host logic of bench.py (CPU): the profiled counter figures apply only to
the grid and kernel sources they were taken on, the VALU figures follow from
their definitions, and a multi-GPU request is refused."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_counter_figures_only_for_the_profiled_grid_and_sources(monkeypatch):
    k = "k_step<double,double,0>"
    e = bench.pmc_entry(k, 4096, 4096)
    assert e is not None and e["sources"] == bench._sources_digest()
    assert bench.pmc_entry(k, 4096, 2048) is None
    assert bench.pmc_entry("k_step<double,double,1>", 4096, 4096) is None
    assert bench.measured_traffic(k, 4096, 4096) == e["fetch_bytes"] + e["write_bytes"]
    # any change of a profiled source voids the figures
    changed = dict(bench._sources_digest())
    changed["csrc/fvna_step.hpp"] = "0" * 64
    monkeypatch.setattr(bench, "_sources_digest", lambda: changed)
    assert bench.pmc_entry(k, 4096, 4096) is None and bench.measured_traffic(k, 4096, 4096) is None
    assert bench.measured_valu(k, 4096, 4096, 2.5e-4) is None


def test_valu_figures_follow_their_definitions():
    k = "k_step<double,double,0>"
    e = bench.pmc_entry(k, 4096, 4096)
    kernel_s = 2.5e-4
    v = bench.measured_valu(k, 4096, 4096, kernel_s)
    cells = 4096 * 4096
    rate = e["valu_lane_ops_per_cell"] * cells / kernel_s
    assert v["lane_ops_per_cell"] == e["valu_lane_ops_per_cell"]
    assert v["frac"] == pytest.approx(rate / (256 * 64 * 2.4e9), abs=1e-4)
    assert v["issue_frac"] == pytest.approx(e["valu_issue_cycles_per_cell"] * cells / kernel_s / (1024 * 2.4e9),
                                            abs=1e-4)
    # issue cycles count every transcendental at its cost: at least the
    # instructions' own cycles (4 lane-cycles of a 16-lane SIMD per wave64 op)
    assert e["valu_issue_cycles_per_cell"] >= e["valu_lane_ops_per_cell"] / 16


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU only" in (r.stdout + r.stderr)

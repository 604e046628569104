"""CPU checks of bench.py's host logic: the one-GPU guard, the roofline of
the dominant kernel, the traffic table's tie to the kernel source, and the
median of the repeated timing passes."""
from __future__ import annotations

import os
import subprocess
import sys

import bench

HERE = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(HERE, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_roofline_picks_the_dominant_kernel_and_prices_its_algorithmic_bytes():
    n = 256
    # (total ms over the timed steps, launches)
    kern = {"cfl": (0.3, 20), "fluid_x": (14.0, 40), "fluid_y": (15.0, 40), "fluid_z": (14.5, 40),
            "ct_x": (12.0, 40), "ct_y": (11.0, 40), "ct_z": (10.0, 40)}
    dom, roof = bench.roofline(kern, n ** 3, 8, n)
    assert dom == "fluid_y" and roof["kernel"] == "fluid_y"
    per_launch = 13 * n ** 3 * 8
    assert roof["bytes_per_launch"] == per_launch
    assert abs(roof["achieved"] - per_launch / (15.0 / 40 / 1e3) / 1e9) < 0.1
    assert abs(roof["frac"] - roof["achieved"] / 8000.0) < 1e-4
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    # kinds that never ran are not candidates
    kern = {"cfl": (0.0, 0), "fluid_x": (1.0, 2), "fluid_y": (0.0, 0), "fluid_z": (0.0, 0),
            "ct_x": (0.5, 2), "ct_y": (0.4, 2), "ct_z": (0.4, 2)}
    assert bench.roofline(kern, 4096, 4, 4096)[0] == "fluid_x"


def test_traffic_is_reported_only_for_the_profiled_source(tmp_path, monkeypatch):
    # a table written for the current kernel source is read back
    table = tmp_path / "traffic.txt"
    table.write_text("# header\nsource_sha256 %s\nf64 fluid_y 1500000000 700000000\n" % bench.kernel_fingerprint())
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(table))
    assert bench.measured_traffic("f64", "fluid_y", 256) == 2200000000
    assert bench.measured_traffic("f64", "ct_y", 256) is None
    # other workloads have no table
    assert bench.measured_traffic("f64", "fluid_y", 128) is None
    # a changed kernel source invalidates it
    src = tmp_path / "k.h"
    src.write_bytes(b"// another kernel source\n")
    monkeypatch.setattr(bench, "KERNEL_SOURCES", (str(src),) + tuple(bench.KERNEL_SOURCES[1:]))
    assert bench.measured_traffic("f64", "fluid_y", 256) is None


def test_repeat_summary_reports_the_median_pass():
    s = bench.repeat_summary([0.071, 0.070, 0.090, 0.069, 0.072], 20)
    assert s["passes"] == 5 and s["steps_each"] == 20
    assert s["median_ms_per_step"] == 3.55   # 0.071 s over 20 steps
    assert s["min_ms_per_step"] == 3.45 and s["max_ms_per_step"] == 4.5
    assert bench.repeat_summary([0.07, 0.08], 10)["median_ms_per_step"] == 7.5
    assert bench.repeat_summary([], 20) is None

"""Host-side logic of bench.py (no GPU): the one-GPU guard, the problem
filter, the clock sampler without a device, and the guard that keeps a
stale counter summary out of the roofline."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_problem_filter_keeps_named_problems():
    probs, desc = bench.make_problems("c1", "square256_NN")
    assert [p.label for p in probs] == ["square256_NN"]
    assert "only square256_NN" in desc
    with pytest.raises(SystemExit):
        bench.make_problems("c1", "no_such_problem")


def test_clock_sampler_without_device_reports_none():
    with bench.ClockSampler(period=0.01) as c:
        pass
    s = c.summary()
    assert set(s) >= {"sclk_mhz", "socket_power_w", "ppt_residency"}
    if s["sclk_mhz"] is None:
        assert "note" in s


def test_kernel_hash_covers_every_kernel_source():
    csrc = os.path.join(ROOT, "paper_1608_05265_amd", "csrc")
    # every sgemm kernel source (the probe library, the dgemm path and the
    # LU driver are separate programs that only call the sgemm kernels)
    kernels = {f for f in os.listdir(csrc) if f.endswith((".hip", ".hpp")) and
               not f.startswith(("probe_", "dgemm", "lu."))}
    assert kernels == set(bench.KERNEL_SOURCES)
    # the tile schedule (choice, order, batch tile lists) is hashed too
    assert "api.cpp" in bench.SCHEDULE_SOURCES


def test_stale_traffic_is_not_reported(tmp_path, monkeypatch):
    h = bench.kernel_sources_hash()
    f = tmp_path / "counters.txt"
    f.write_text("traffic_bytes_per_launch fp32 %s 123.0\n"
                 "traffic_bytes_per_launch bf16x3 0000000000000000 456.0\n" % h)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("fp32") == 123.0
    assert bench.measured_traffic("bf16x3") is None
    assert bench.measured_traffic("other") is None

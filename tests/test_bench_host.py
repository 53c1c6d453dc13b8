"""Host-side contracts of the benchmark (no GPU): the one-GPU refusal, and
the HBM traffic of the cell kernel reported from the committed counter
profile only while the kernel source is the one the counters were taken on."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_reported_only_for_the_profiled_kernel_source(monkeypatch):
    import bench
    text = open(os.path.join(ROOT, "profiles", "k_cell_gemm-si30-24c.md")).read()
    m = re.search(r"pmc-traffic: kernel=k_cell_gemm bytes_per_launch=(\d+) "
                  r"source_sha256=([0-9a-f]+)", text)
    assert m, "machine-readable traffic line missing"
    # at least the method's minimum for one colour launch on the 30-atom
    # workload (cell matrices + vectors once: ~0.89 GB)
    assert int(m.group(1)) > 0.89e9
    if m.group(2) == bench.cell_kernel_source_hash():
        assert bench.measured_traffic() == int(m.group(1))
    else:                                   # kernel changed since the counters
        assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "cell_kernel_source_hash", lambda: "0" * 64)
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "cell_kernel_source_hash", lambda: m.group(2))
    assert bench.measured_traffic() == int(m.group(1))

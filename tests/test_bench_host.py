"""Host-side contracts of the benchmark (no GPU): the one-GPU refusal, and
that the committed counter profile of the cell kernel was taken on the
committed kernel source (the benchmark reports its HBM traffic only then)."""
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


def test_traffic_profile_matches_the_kernel_source():
    import bench
    text = open(os.path.join(ROOT, "profiles", "k_cell_gemm-si30-24c.md")).read()
    m = re.search(r"pmc-traffic: kernel=k_cell_gemm bytes_per_launch=(\d+) "
                  r"source_sha256=([0-9a-f]+)", text)
    assert m, "machine-readable traffic line missing"
    assert m.group(2) == bench.cell_kernel_source_hash()
    assert bench.measured_traffic() == int(m.group(1))
    # the per-launch bytes are at least the method's minimum for one colour
    # launch on the 30-atom workload (cell matrices + vectors once: ~0.89 GB)
    assert int(m.group(1)) > 0.89e9

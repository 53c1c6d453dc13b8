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


def _undefined_globals(path):
    """Names a function of the file reads as globals that the module never
    binds and that are not builtins (what would raise NameError only when
    that code path runs)."""
    import builtins
    import symtable
    src = open(path).read()
    top = symtable.symtable(src, path, "exec")
    bound = {s.get_name() for s in top.get_symbols() if s.is_assigned() or s.is_imported()}
    bound |= set(dir(builtins)) | {"__file__", "__name__"}
    missing = set()

    def walk(t):
        for ch in t.get_children():
            if ch.get_type() == "function":
                for s in ch.get_symbols():
                    if s.is_global() and s.is_referenced() and s.get_name() not in bound:
                        missing.add((ch.get_name(), s.get_name()))
            walk(ch)
    walk(top)
    return missing


def test_host_scripts_bind_every_name_they_use():
    """bench.py, the binding, the learned-bounds driver, the generators and
    the oracle: every name a function reads is bound somewhere (a local import in an enclosing scope
    counts), so the rarely run modes fail on their arithmetic, not on a
    missing import."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    import glob
    rels = ["bench.py", "__graft_entry__.py",
            os.path.join("paper_1610_02121_amd", "binding.py"),
            os.path.join("paper_1610_02121_amd", "learned.py")]
    for d in ("synth", "oracle"):
        rels += sorted(os.path.relpath(f, root) for f in glob.glob(os.path.join(root, d, "*.py")))
    for rel in rels:
        missing = _undefined_globals(os.path.join(root, rel))
        assert not missing, (rel, sorted(missing))

"""Host-side parts of bench.py: the one-GPU refusal and the gate that keeps a
committed HBM-traffic figure only while the kernel sources it was measured on
are unchanged."""
import hashlib
import importlib.util
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ("paper_2306_06795_amd/csrc/kernels.hpp", "paper_2306_06795_amd/csrc/mas.hip")


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_line_is_used_only_for_its_workload_and_sources(tmp_path):
    for fn in SOURCES:
        os.makedirs(tmp_path / os.path.dirname(fn), exist_ok=True)
        shutil.copy(os.path.join(ROOT, fn), tmp_path / fn)
    h = hashlib.sha256()
    for fn in SOURCES:
        h.update((tmp_path / fn).read_bytes())
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k.md").write_text(
        "# summary\n\ntraffic: workload=w1 precision=fp64 relax=vanka kind=tpp bytes_per_launch=1234 "
        f"sources={h.hexdigest()}\n")
    b = _bench()
    b.ROOT = str(tmp_path)
    assert b.measured_traffic("w1", "fp64", "vanka", "tpp") == 1234.0
    assert b.measured_traffic("w1", "fp32", "vanka", "tpp") is None
    assert b.measured_traffic("w1", "fp64", "dlsc", "tpp") is None
    assert b.measured_traffic("w1", "fp64", "vanka", "generic") is None
    assert b.measured_traffic("w2", "fp64", "vanka", "tpp") is None
    # any change to the kernel sources voids the figure
    with open(tmp_path / SOURCES[0], "a") as f:
        f.write("\n")
    assert b.measured_traffic("w1", "fp64", "vanka", "tpp") is None

"""Host-side logic of bench.py (no GPU): the refusal of several GPUs, and the lookup of
the measured HBM traffic, which must be ignored once the kernel sources differ from the
profiled ones."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def _tree(tmp_path):
    """A copy of the files the traffic lookup reads: the profile and the kernel sources."""
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1903_06479_amd" / "csrc").mkdir(parents=True)
    shutil.copy(os.path.join(ROOT, "profiles", "step_kernel_throughput_100k_642.md"), tmp_path / "profiles")
    for f in ("npfem_kernels.hip", "npfem_internal.h"):
        shutil.copy(os.path.join(ROOT, "paper_1903_06479_amd", "csrc", f), tmp_path / "paper_1903_06479_amd" / "csrc")
    return tmp_path


def test_measured_traffic_is_tied_to_the_profiled_sources(tmp_path, monkeypatch):
    import bench
    prof = open(os.path.join(ROOT, "profiles", "step_kernel_throughput_100k_642.md")).read()
    if "traffic_bytes_per_launch:" not in prof:
        pytest.skip("no traffic figure in the committed profile")
    tree = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tree))
    want = float(prof.split("traffic_bytes_per_launch:")[1].split()[0])
    got = bench.measured_traffic()
    if got is None:
        pytest.skip("the committed profile predates the current kernel sources")
    assert got == pytest.approx(want)
    # any change to the kernel sources invalidates the figure
    k = tree / "paper_1903_06479_amd" / "csrc" / "npfem_kernels.hip"
    k.write_text(k.read_text() + "\n")
    assert bench.measured_traffic() is None
    # and so does a missing profile
    os.remove(tree / "profiles" / "step_kernel_throughput_100k_642.md")
    assert bench.measured_traffic() is None

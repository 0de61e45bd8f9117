"""bench.py's host logic (no GPU): the one-GPU contract, the per-site byte
counts behind the roofline, and the rule that the HBM traffic figure is
reported only while the committed counter summary matches the kernel
source."""
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
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_site():
    # 37 populations read and 37 written per site update
    assert bench.bytes_per_site("f64") == 592
    assert bench.bytes_per_site("f32dev") == 296


def test_traffic_only_for_the_profiled_source(monkeypatch):
    path = os.path.join(ROOT, "profiles", "step_f64_rt3_4096x12288_counters.txt")
    text = open(path).read()
    sha = text.split("kernel_source_sha:")[1].split()[0]
    monkeypatch.setattr(bench, "step_source_hash", lambda: sha)
    b = bench.measured_traffic("rt3_4096x12288", "f64")
    alg = 592 * 4096 * 12288
    assert b is not None and alg <= b <= 1.1 * alg
    monkeypatch.setattr(bench, "step_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("rt3_4096x12288", "f64") is None
    assert bench.measured_traffic("no_such_workload", "f64") is None


@pytest.mark.parametrize("name", ["step.hip", "common.h", "lattice_constants.h"])
def test_source_hash_covers_the_step_sources(name, monkeypatch, tmp_path):
    """Changing the code of any file the step kernel is built from changes
    the hash; a comment or a blank line does not."""
    csrc = tmp_path / "paper_1405_1253_amd" / "csrc"
    csrc.mkdir(parents=True)
    for n in ("step.hip", "common.h", "lattice_constants.h"):
        (csrc / n).write_bytes(open(os.path.join(ROOT, "paper_1405_1253_amd", "csrc", n), "rb").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.step_source_hash()
    assert h0 == bench.step_source_hash()
    with open(csrc / name, "a") as fh:
        fh.write("\n// a comment\n/* another\n   comment */\n\n")
    assert bench.step_source_hash() == h0
    with open(csrc / name, "a") as fh:
        fh.write("static int extra_symbol;\n")
    assert bench.step_source_hash() != h0


def test_adjoint_traffic_only_for_the_profiled_source(monkeypatch):
    path = os.path.join(ROOT, "profiles", "adjoint_f32_rt3_2048x6144_counters.txt")
    sha = open(path).read().split("adjoint_source_sha:")[1].split()[0]
    monkeypatch.setattr(bench, "adjoint_source_hash", lambda: sha)
    b = bench.measured_adjoint_traffic("rt3_2048x6144_adj")
    alg = (37 * 4 + 4 * 4 + 37 * 4) * 2048 * 6144      # float lam in and out, float moments
    assert b is not None and alg <= b <= 1.1 * alg
    assert bench.measured_adjoint_traffic("rt3_512x1536_adj") is None      # not profiled
    monkeypatch.setattr(bench, "adjoint_source_hash", lambda: "0" * 16)
    assert bench.measured_adjoint_traffic("rt3_2048x6144_adj") is None

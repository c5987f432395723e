"""Host logic of bench.py (no GPU): the one-GPU contract and the profile
lookup that feeds the roofline's measured traffic."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_profile_hash_covers_sources_and_flags(monkeypatch):
    from paper_1704_02724_amd import build
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()
    monkeypatch.setattr(build, "HIPCC_FLAGS", build.HIPCC_FLAGS + ["-DSOMETHING_ELSE"])
    assert bench.kernel_source_hash() != h


def test_profiled_counts_only_for_the_profiled_kernel(monkeypatch):
    path = os.path.join(ROOT, "profiles", "k_cast_fp32_rebased_depth24.md")
    if not os.path.exists(path):
        pytest.skip("no committed profile")
    with open(path) as f:
        text = f.read()
    profiled = next(l.split(":", 1)[1].strip() for l in text.splitlines()
                    if l.startswith("kernel_source_sha256_16"))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: profiled)
    traffic, valu = bench.profiled_counts("fp32_rebased", "depth24")
    assert traffic > 0 and valu > 0
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.profiled_counts("fp32_rebased", "depth24") == (None, None)
    assert bench.profiled_counts("fp32_rebased", "no_such_workload") == (None, None)

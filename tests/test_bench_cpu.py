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


def test_roofline_bound_follows_the_counters():
    """The bound is the larger of the two measured fractions (vector issue
    against its peak, HBM bytes against 8 TB/s); both null without a
    matching profile."""
    t = 1e-3  # one launch of 1 ms
    issue_bound = bench.roofline(8e9, t, 0.4e9, 0.6e9, 5e12)
    assert issue_bound["bound"] == "alu"
    assert issue_bound["frac"] == round(0.6e9 / t / bench.VALU_PEAK, 4)
    assert issue_bound["peak"] == round(bench.VALU_PEAK / 1e9, 1)
    assert issue_bound["hbm_measured_frac"] == round(0.4e9 / t / bench.HBM_PEAK, 4)
    assert issue_bound["alg_bytes_frac"] == round(8e9 / t / bench.HBM_PEAK, 4)
    hbm_bound = bench.roofline(8e9, t, 7.9e9, 0.1e9, 5e12)
    assert hbm_bound["bound"] == "hbm" and hbm_bound["unit"] == "GB/s"
    assert hbm_bound["frac"] == round(7.9e9 / t / bench.HBM_PEAK, 4)
    none = bench.roofline(8e9, t, None, None, None)
    assert none["bound"] is None and none["frac"] is None and none["traffic"] is None
    assert none["alg_bytes_frac"] == round(8e9 / t / bench.HBM_PEAK, 4)

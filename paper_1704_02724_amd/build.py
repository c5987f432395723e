"""Build step for libcvx: compiles the HIP sources for gfx950 into lib/libcvx.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "lib")
LIB_PATH = os.path.join(LIB_DIR, "libcvx.so")
SOURCES = ["cvx_api.cpp", "cvx_validate.cpp", "cvx_upload.hip", "cvx_cast.hip",
           "cvx_stroke.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no implicit contraction: every fused multiply-add is written in the
    # source, so all kernel instances round identically
    "-ffp-contract=off",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # machine-level loop-invariant code motion lifts constants of the per-ray
    # setup out of the persistent tile loop, where they stay live through the
    # whole traversal; without it the FP32 render kernel needs 61 VGPRs
    # instead of 64 (earlier versions of the loop spilled 8-12 bytes per lane
    # with it) and keeps the same hot-loop instructions
    "-mllvm", "-disable-machine-licm",
    # the render loop is bound by vector instruction issue; the scheduler's
    # ILP strategy orders its independent instructions so that more of them
    # issue back to back (same instructions, same registers and occupancy;
    # 0.4-1.4 % faster on the depth-24 stereo workload over five interleaved
    # comparisons with the default strategy)
    "-mllvm", "-amdgpu-sched-strategy=max-ilp",
]


# The vector-issue probe behind the caster's roofline (a measurement program,
# not part of the library): lib/probe_valu, run by bench.py --issue-probe.
PROBE_SRC = os.path.join(CSRC, "probe_valu.hip")
PROBE_PATH = os.path.join(LIB_DIR, "probe_valu")
PROBE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    return res


def build(verbose: bool = False) -> str:
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    res = _hipcc(["hipcc"] + HIPCC_FLAGS + ["-I" + os.path.join(ROOT, "include"), "-o", tmp]
                 + [os.path.join(CSRC, s) for s in SOURCES])
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB_PATH)
    ptmp = PROBE_PATH + ".tmp"
    _hipcc(["hipcc"] + PROBE_FLAGS + ["-o", ptmp, PROBE_SRC])
    os.replace(ptmp, PROBE_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))

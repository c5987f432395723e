"""The C-ABI from plain C: tests/capi/cvx_c_check.c includes include/cvx.h
and the HIP runtime header only, links libcvx.so, and renders a canvas whose
image has a closed form (see the program's header).  On the CPU the program
must compile as C99 without warnings; on the GPU it must print "ok"."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "capi", "cvx_c_check.c")
OUT = os.path.join(ROOT, "tests", "capi", "_build", "cvx_c_check")
LIB_DIR = os.path.join(ROOT, "paper_1704_02724_amd", "lib")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


HDR = os.path.join(ROOT, "include", "cvx.h")


def build_c_check():
    """Compile the program with gcc (host code only) if missing or older than
    its source or the header (the structures it passes are the header's)."""
    if not os.path.exists(os.path.join(LIB_DIR, "libcvx.so")):
        pytest.skip("libcvx.so is not built")
    if os.path.exists(OUT) and os.path.getmtime(OUT) >= max(os.path.getmtime(SRC),
                                                            os.path.getmtime(HDR)):
        return OUT
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    cmd = ["gcc", "-std=c99", "-O1", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(ROCM, "include"), SRC,
           "-L" + LIB_DIR, "-lcvx", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath,$ORIGIN/../../../paper_1704_02724_amd/lib",
           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm", "-o", OUT + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    os.replace(OUT + ".tmp", OUT)
    return OUT


def test_c_program_compiles_against_the_header():
    assert os.path.exists(build_c_check())


@pytest.mark.gpu
def test_c_program_renders_the_closed_form():
    exe = build_c_check()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr)
    assert r.stdout.strip().endswith("ok")

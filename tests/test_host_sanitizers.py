"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the CPU
oracle (oracle/oracle.c), the stroke builder (canvasgen/builder.cpp) and the
pool validator of the library (csrc/cvx_validate.cpp) are rebuilt with
-fsanitize=address,undefined and run on seeded inputs in a child process
(tests/sanitize/run_sanitized.py, the ASan runtime preloaded); any sanitizer
report fails the test, and the results must equal those of the normal
builds bit for bit."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
       "-fno-sanitize-recover=undefined", "-fPIC", "-shared", "-pthread"]


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime")
    d = tmp_path_factory.mktemp("san")
    libs = {"oracle": str(d / "liboracle_san.so"), "builder": str(d / "libcanvasgen_san.so"),
            "validate": str(d / "libvalidate_san.so")}
    cmds = [
        ["gcc", "-std=c11", "-ffp-contract=off", "-fno-fast-math"] + SAN +
        ["-o", libs["oracle"], os.path.join(ROOT, "oracle", "oracle.c"), "-lm"],
        ["g++", "-std=c++17"] + SAN + ["-o", libs["builder"],
                                       os.path.join(ROOT, "canvasgen", "builder.cpp")],
        ["g++", "-std=c++17"] + SAN + [
            "-I" + os.path.join(ROOT, "include"),
            "-I" + os.path.join(ROOT, "paper_1704_02724_amd", "csrc"), "-o", libs["validate"],
            os.path.join(ROOT, "tests", "sanitize", "validate_shim.cpp"),
            os.path.join(ROOT, "paper_1704_02724_amd", "csrc", "cvx_validate.cpp")],
    ]
    for c in cmds:
        r = subprocess.run(c, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr
    out = str(d / "san.npz")
    env = dict(os.environ, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitize", "run_sanitized.py"),
                        libs["oracle"], libs["builder"], libs["validate"], out],
                       capture_output=True, text=True, timeout=600, env=env)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    return np.load(out)


def test_oracle_clean_and_unchanged(sanitized):
    from oracle import oracle
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from sanitize.cases import oracle_cases
    for name, (canvases, views) in oracle_cases().items():
        r = oracle.render(canvases, views, max_leaves=64, threads=4)
        for k in ("rgba", "flags", "n_leaves", "leaf_ids", "leaf_len", "alg_bytes"):
            np.testing.assert_array_equal(sanitized[f"oracle_{name}_{k}"], r[k], err_msg=name + k)


def test_builder_clean_and_unchanged(sanitized):
    from sanitize.cases import builder_case
    cv = builder_case()
    np.testing.assert_array_equal(sanitized["builder_nodes"], cv.nodes)
    np.testing.assert_array_equal(sanitized["builder_leaves"], cv.leaves.view(np.uint8))


def test_validator_clean_and_unchanged(sanitized):
    from paper_1704_02724_amd import cvx
    from sanitize.cases import validate_cases
    codes = []
    for desc, nodes, leaves in validate_cases():
        d = cvx.make_desc(tuple(desc.origin), desc.root_edge, desc.R, desc.max_depth,
                          desc.leaf_format)
        codes.append(cvx.cvx_validate_pool(d, nodes, leaves)[0])
    assert codes[0] == 0 and all(c != 0 for c in codes[1:])
    np.testing.assert_array_equal(sanitized["validate_codes"], np.array(codes))

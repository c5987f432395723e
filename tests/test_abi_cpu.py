"""The C-ABI library without a GPU: symbols, host validation, error strings."""
import re
import os

import numpy as np
import pytest

from canvasgen import LEAF, LEAF_F64, LEAF_RGBA8_F16, NONE, make_view
from canvasgen import trees

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cvx():
    from paper_1704_02724_amd import cvx as mod
    return mod


def test_exports_every_declared_symbol(cvx):
    hdr = open(os.path.join(ROOT, "include", "cvx.h")).read()
    declared = set(re.findall(r"^[\w \*]+?\b(cvx_\w+)\(", hdr, flags=re.M))
    assert {"cvx_create", "cvx_upload_pool", "cvx_render", "cvx_destroy"} <= declared
    lib = cvx.library()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(cvx.EXPORTED)


def test_status_strings(cvx):
    assert cvx.status_name(0) == "CVX_OK"
    assert cvx.status_name(-2) == "CVX_ERR_BAD_POOL"
    assert cvx.status_name(-99) == "CVX_ERR_UNKNOWN"


def _desc(cvx, cv, **over):
    d = dict(origin=cv.origin, root_edge=cv.root_edge, R=cv.R, max_depth=cv.max_depth,
             leaf_format=cv.leaf_format)
    d.update(over)
    return cvx.make_desc(d["origin"], d["root_edge"], d["R"], d["max_depth"], d["leaf_format"])


def test_valid_pool_accepted(cvx):
    for fmt in (LEAF_F64, LEAF_RGBA8_F16):
        cv = trees.random_tree(2, 5, seed=3, leaf_format=fmt)
        rc, msg = cvx.cvx_validate_pool(_desc(cvx, cv), cv.nodes, cv.leaves)
        assert rc == 0, msg


def _corrupt_cases(cv):
    n = cv.nodes
    g = int(n[0, 0])                 # first child group of the root
    leaf_node = next(i for i in range(g, len(n)) if n[i, 0] & LEAF)
    inner = next(i for i in range(g, len(n)) if not n[i, 0] & LEAF)
    cases = {}
    a = n.copy(); a[0, 0] = len(n) + 8; cases["child out of range"] = a
    a = n.copy(); a[0, 0] = g + 3; cases["child not 8-aligned"] = a
    a = n.copy(); a[inner, 0] = g; cases["group reached twice (cycle)"] = a
    a = n.copy(); a[g + 2, 1] = 0 if n[g + 2, 1] != 0 else 1; cases["parent mismatch"] = a
    a = n.copy(); a[leaf_node, 0] = LEAF | len(cv.leaves); cases["leaf index out of range"] = a
    a = n.copy(); a[0, 1] = 5; cases["root with a parent"] = a
    a = n.copy(); a[0, 0] = 0; cases["child group inside the root array"] = a
    return cases


def test_corrupt_pools_rejected(cvx):
    cv = trees.random_tree(1, 5, seed=4, leaf_format=LEAF_RGBA8_F16)
    d = _desc(cvx, cv)
    for name, nodes in _corrupt_cases(cv).items():
        rc, msg = cvx.cvx_validate_pool(d, nodes, cv.leaves)
        assert rc == cvx.CVX_ERR_BAD_POOL, (name, rc, msg)
        assert msg


def test_depth_limit_and_desc_checks(cvx):
    cv = trees.random_tree(1, 6, seed=5, leaf_format=LEAF_RGBA8_F16)
    real_depth = 6
    rc, msg = cvx.cvx_validate_pool(_desc(cvx, cv, max_depth=real_depth - 1), cv.nodes, cv.leaves)
    assert rc == cvx.CVX_ERR_BAD_POOL and "depth" in msg
    for over in (dict(R=0), dict(max_depth=31), dict(root_edge=0.0), dict(leaf_format=2),
                 dict(root_edge=float("nan")), dict(R=4, max_depth=30),
                 dict(R=2, max_depth=30)):
        rc, msg = cvx.cvx_validate_pool(_desc(cvx, cv, **over), cv.nodes, cv.leaves)
        assert rc == cvx.CVX_ERR_INVALID_ARG, (over, rc, msg)


def test_bad_leaf_payloads(cvx):
    cv = trees.random_tree(1, 3, seed=6, leaf_format=LEAF_RGBA8_F16)
    lv = cv.leaves.copy(); lv["kappa"][0] = 0xBC00          # -1.0 in half
    assert cvx.cvx_validate_pool(_desc(cvx, cv), cv.nodes, lv)[0] == cvx.CVX_ERR_BAD_POOL
    lv = cv.leaves.copy(); lv["kappa"][1] = 0x7C00          # +inf
    assert cvx.cvx_validate_pool(_desc(cvx, cv), cv.nodes, lv)[0] == cvx.CVX_ERR_BAD_POOL
    cf = trees.random_tree(1, 3, seed=6, leaf_format=LEAF_F64)
    lf = cf.leaves.copy(); lf["kappa"][2] = np.nan
    assert cvx.cvx_validate_pool(_desc(cvx, cf), cf.nodes, lf)[0] == cvx.CVX_ERR_BAD_POOL


def test_view_validation(cvx):
    cv = trees.random_tree(1, 3, seed=7, leaf_format=LEAF_RGBA8_F16)
    d = _desc(cvx, cv)
    good = make_view((0.5, 0.5, -1.0), (0.0, 0.0, 1.0), 0.5, 8, 8)
    assert cvx.cvx_validate_views(cvx.make_views([good]), [d])[0] == 0
    bads = [dict(good, W=0), dict(good, H=0), dict(good, canvas_id=1), dict(good, canvas_id=-1),
            dict(good, tan_x=0.0), dict(good, alpha_stop=0.0),
            dict(good, up=(0.0, 0.9, 0.0)), dict(good, right=(1.0, 0.0, 0.1)),
            dict(good, eye=(float("inf"), 0.0, 0.0))]
    for b in bads:
        rc, msg = cvx.cvx_validate_views(cvx.make_views([b]), [d])
        assert rc == cvx.CVX_ERR_INVALID_ARG, (b, rc)
    rc, _ = cvx.cvx_validate_views(cvx.make_views([dict(good, canvas_id=1)]), [d, None])
    assert rc == cvx.CVX_ERR_INVALID_ARG


def test_create_without_gpu_fails_cleanly(cvx):
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(cvx.CvxError):
        cvx.cvx_create(0, 0)


def test_binding_constants_match_the_header(cvx):
    hdr = open(os.path.join(ROOT, "include", "cvx.h")).read()
    defines = re.findall(r"^#define (CVX_\w+) \(?(-?(?:0x[0-9a-fA-F]+|\d+))u?\)?", hdr,
                         flags=re.M)
    assert len(defines) > 20
    missing = [n for n, _ in defines if not hasattr(cvx, n)]
    assert not missing, missing
    for name, value in defines:
        assert getattr(cvx, name) == int(value, 0), name


def test_binding_fails_loudly_without_the_library():
    """No fallback: with libcvx.so absent the binding (and so the session,
    the tests and the benchmark) cannot be imported."""
    import subprocess
    import sys
    code = ("import paper_1704_02724_amd.build as b; b.LIB_PATH = '/nonexistent/libcvx.so'; "
            "import paper_1704_02724_amd.cvx")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "/nonexistent/libcvx.so is not built" in r.stderr


def test_binding_struct_layouts_match_the_header(cvx, tmp_path):
    """Every ctypes structure of the binding has the C header's size and
    field offsets (a C program compiled against include/cvx.h prints them)."""
    import ctypes
    import subprocess
    structs = ["cvx_canvas_desc", "cvx_view", "cvx_trace", "cvx_render_opts", "cvx_tune_result",
               "cvx_edit", "cvx_stroke"]
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "cvx.h"', "int main(void) {"]
    for name in structs:
        lines.append(f'  printf("{name} sizeof %zu\\n", sizeof({name}));')
        for field, _ in getattr(cvx, name)._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(ROOT, "include")
    subprocess.check_call(["gcc", "-std=c99", "-I", inc, "-o", str(exe), str(src)])
    c = {}
    for ln in subprocess.check_output([str(exe)], text=True).splitlines():
        name, field, value = ln.split()
        c[(name, field)] = int(value)
    for name in structs:
        st = getattr(cvx, name)
        assert ctypes.sizeof(st) == c[(name, "sizeof")], name
        for field, _ in st._fields_:
            assert getattr(st, field).offset == c[(name, field)], (name, field)

"""Child process of tests/test_host_sanitizers.py: runs the host libraries
built with AddressSanitizer and UndefinedBehaviorSanitizer (paths in argv)
on small seeded inputs and saves the results for comparison with the normal
builds.  Usage: run_sanitized.py ORACLE_SO BUILDER_SO VALIDATE_SO OUT_NPZ"""
import ctypes
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE)]

import numpy as np  # noqa: E402

import canvasgen.pool as pool  # noqa: E402
from oracle import oracle  # noqa: E402

from sanitize.cases import builder_case, oracle_cases, validate_cases  # noqa: E402

oracle_so, builder_so, validate_so, out = sys.argv[1:5]
oracle.LIB, oracle._lib = oracle_so, None
pool.LIB_PATH, pool._lib = builder_so, None

res = {}
for name, (canvases, views) in oracle_cases().items():
    r = oracle.render(canvases, views, max_leaves=64, threads=4)
    for k in ("rgba", "flags", "n_leaves", "leaf_ids", "leaf_len", "alg_bytes"):
        res[f"oracle_{name}_{k}"] = r[k]
cv = builder_case()
res["builder_nodes"] = cv.nodes
res["builder_leaves"] = cv.leaves.view(np.uint8)

lib = ctypes.CDLL(validate_so)
vp = ctypes.c_void_p
lib.san_validate_pool.argtypes = [vp, vp, ctypes.c_uint64, vp, ctypes.c_uint64]
lib.san_validate_pool.restype = ctypes.c_int
codes = []
for desc, nodes, leaves in validate_cases():
    codes.append(lib.san_validate_pool(ctypes.byref(desc), nodes.ctypes.data, nodes.size // 2,
                                       leaves.ctypes.data if leaves.size else None, len(leaves)))
res["validate_codes"] = np.array(codes)
np.savez(out, **res)
print("sanitized run done")

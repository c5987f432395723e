"""Seeded inputs shared by the sanitized and the normal runs of the host
libraries (oracle renders, one stroke build, valid and corrupt pools)."""
import ctypes

import numpy as np

from canvasgen import LEAF_F64, LEAF_RGBA8_F16, trees
from canvasgen.pool import build_from_strokes
from canvasgen.strokes import gen_strokes
from helpers import random_rays, ray_views


def oracle_cases():
    out = {}
    for R, depth, seed in [(1, 6, 1), (2, 5, 2), (3, 4, 3)]:
        cv = trees.random_tree(R, depth, seed=seed, max_nodes=3000, leaf_format=LEAF_F64)
        rng = np.random.Generator(np.random.PCG64(seed))
        out[f"r{R}d{depth}"] = ([cv], ray_views(*random_rays(rng, 200, R=float(R))))
    return out


def builder_case():
    st = gen_strokes(np.random.Generator(np.random.PCG64(21)), 24, -8.0, -4.0)
    return build_from_strokes(st, 1, 12, 4.0, LEAF_RGBA8_F16, split_depth=3, threads=4)


def validate_cases():
    """(desc, nodes, leaves): a valid pool and the corrupt variants of the
    ABI tests."""
    from test_abi_cpu import _corrupt_cases
    cv = trees.random_tree(1, 5, seed=4, leaf_format=LEAF_RGBA8_F16)
    desc = make_desc(cv.origin, cv.root_edge, cv.R, cv.max_depth, cv.leaf_format)
    cases = [(desc, cv.nodes, cv.leaves)]
    for nodes in _corrupt_cases(cv).values():
        cases.append((desc, np.ascontiguousarray(nodes, np.uint32), cv.leaves))
    short = make_desc(cv.origin, cv.root_edge, cv.R, cv.max_depth - 1, cv.leaf_format)
    cases.append((short, cv.nodes, cv.leaves))
    return cases


class Desc(ctypes.Structure):
    """cvx_canvas_desc of include/cvx.h (declared here so that the sanitized
    run loads no GPU library)."""
    _fields_ = [("origin", ctypes.c_double * 3), ("root_edge", ctypes.c_double),
                ("R", ctypes.c_uint32), ("max_depth", ctypes.c_uint32),
                ("leaf_format", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


def make_desc(origin, root_edge, R, max_depth, leaf_format):
    return Desc((ctypes.c_double * 3)(*origin), root_edge, R, max_depth, leaf_format, 0)

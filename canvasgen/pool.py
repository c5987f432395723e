"""Node-pool container and the native stroke builder binding (input generation).

A canvas is an array of R^3 octree roots (Sec. 4) stored as pointer-free
linear pools indexed by cell id (Sec. 4.1.1): ``nodes`` holds {child, parent}
per cell, 8 children are consecutive and only the first is stored.  A leaf
has bit 31 set in ``child`` and the low bits index ``leaves``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

LEAF = 0x80000000
NONE = 0xFFFFFFFF

LEAF_RGBA8_F16 = 0
LEAF_F64 = 1

LEAF_DTYPE = {
    LEAF_RGBA8_F16: np.dtype([("r", "u1"), ("g", "u1"), ("b", "u1"), ("a", "u1"),
                              ("kappa", "<u2"), ("pad", "<u2")]),
    LEAF_F64: np.dtype([("r", "<f8"), ("g", "<f8"), ("b", "<f8"), ("kappa", "<f8")]),
}

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcanvasgen.so")


class Canvas:
    """A canvas ready for upload: desc + nodes (n,2) uint32 + leaves (structured)."""

    def __init__(self, nodes, leaves, R, max_depth, leaf_format, origin=(0.0, 0.0, 0.0),
                 root_edge=None, stats=None):
        self.nodes = np.ascontiguousarray(nodes, dtype=np.uint32).reshape(-1, 2)
        self.leaves = np.ascontiguousarray(leaves)
        assert self.leaves.dtype == LEAF_DTYPE[leaf_format]
        self.R = int(R)
        self.max_depth = int(max_depth)
        self.leaf_format = int(leaf_format)
        self.origin = tuple(float(v) for v in origin)
        self.root_edge = float(1.0 / R if root_edge is None else root_edge)
        self.stats = dict(stats or {})

    @property
    def n_nodes(self):
        return len(self.nodes)

    @property
    def n_leaves(self):
        return len(self.leaves)

    def desc(self):
        return dict(origin=self.origin, root_edge=self.root_edge, R=self.R,
                    max_depth=self.max_depth, leaf_format=self.leaf_format)


def build_lib(force: bool = True) -> str:
    """Compile the stroke builder with g++ (host code only)."""
    src = os.path.join(_HERE, "builder.cpp")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, src])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_lib(force=False)
        lib = ctypes.CDLL(LIB_PATH)
        u32, u64, i32, f64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        lib.cg_build.argtypes = [u32, u32, f64, u32, i32, i32, vp, vp, vp, vp, vp, i32,
                                 ctypes.POINTER(vp)]
        lib.cg_build.restype = i32
        lib.cg_result_sizes.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        lib.cg_emit.argtypes = [vp, vp, vp, vp, ctypes.POINTER(u32), i32]
        lib.cg_emit.restype = i32
        lib.cg_result_free.argtypes = [vp]
        lib.cg_set_verbose.argtypes = [i32]
        lib.cg_set_verbose.restype = None
        lib.cg_f32_to_f16.argtypes = [ctypes.c_float]
        lib.cg_f32_to_f16.restype = ctypes.c_uint16
        _lib = lib
    return _lib


def f32_to_f16_bits(x: float) -> int:
    return int(_load().cg_f32_to_f16(float(x)))


def build_from_strokes(strokes, R: int, max_depth: int, k: float, leaf_format: int,
                       split_depth: int = 0, threads: int = 0, verbose: bool = False) -> Canvas:
    """Refine and paint the canvas stroke by stroke (Sec. 5.1-5.2), emit the pool.
    verbose: the builder prints progress lines on stderr (long builds)."""
    lib = _load()
    lib.cg_set_verbose(1 if verbose else 0)
    if threads <= 0:
        threads = min(16, os.cpu_count() or 1)
    h = ctypes.c_void_p()
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    rc = lib.cg_build(R, max_depth, float(k), split_depth, threads, strokes.n,
                      ptr(strokes.stamp_off), ptr(strokes.stamps), ptr(strokes.rgb),
                      ptr(strokes.sigma), ptr(strokes.radius), leaf_format, ctypes.byref(h))
    if rc != 0:
        raise RuntimeError(f"canvas builder failed with code {rc}")
    try:
        nn, nl, md = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint32()
        lib.cg_result_sizes(h, ctypes.byref(nn), ctypes.byref(nl))
        nodes = np.empty((nn.value, 2), np.uint32)
        leaves = np.empty(nl.value, LEAF_DTYPE[leaf_format])
        hist = np.zeros(64, np.uint64)
        rc = lib.cg_emit(h, ptr(nodes), ptr(leaves), ptr(hist), ctypes.byref(md), threads)
        if rc != 0:
            raise RuntimeError(f"canvas builder emission failed with code {rc}")
    finally:
        lib.cg_result_free(h)
    stats = dict(max_depth_seen=int(md.value), leaf_depth_hist=hist[:md.value + 1].tolist(),
                 k=float(k), n_strokes=strokes.n)
    return Canvas(nodes, leaves, R, max_depth, leaf_format, stats=stats)

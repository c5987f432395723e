"""Python binding of the CPU FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  It depends only on the
canvas and view descriptions (plain arrays), not on the GPU package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

FLAG_NEAR_FACE = 1
FLAG_TERM_AMBIG = 2
FLAG_STEP_CAP = 4
FLAG_BAD_POOL = 8

EPS_FACE = 1e-12


class _Canvas(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("root_edge", ctypes.c_double),
                ("R", ctypes.c_uint32), ("max_depth", ctypes.c_uint32),
                ("leaf_format", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("nodes", ctypes.c_void_p), ("n_nodes", ctypes.c_uint64),
                ("leaves", ctypes.c_void_p), ("n_leaves", ctypes.c_uint64)]


class _View(ctypes.Structure):
    _fields_ = [("canvas", ctypes.c_int32), ("W", ctypes.c_uint32), ("H", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("eye", ctypes.c_double * 3),
                ("right", ctypes.c_double * 3), ("up", ctypes.c_double * 3),
                ("fwd", ctypes.c_double * 3), ("tan_x", ctypes.c_double),
                ("tan_y", ctypes.c_double), ("out_offset_px", ctypes.c_uint64),
                ("alpha_stop", ctypes.c_double)]


def build(force: bool = True) -> str:
    """Compile the oracle: plain C, FP64, no floating-point contraction."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-pthread", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        # CVX_ORACLE_LIB: another build of oracle.c (the mutation check in
        # tests/oracle_mutants.py runs the pins against planted mistakes)
        path = os.environ.get("CVX_ORACLE_LIB") or LIB
        if path == LIB and not os.path.exists(LIB):
            build(force=False)
        lib = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        lib.orc_render.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_uint64,
                                   ctypes.c_double, ctypes.c_uint32, vp, vp, vp, vp, vp, vp, vp,
                                   vp, vp, ctypes.c_int]
        lib.orc_render.restype = ctypes.c_int
        lib.orc_ray_dir.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, vp]
        lib.orc_ray_setup.argtypes = [vp, vp, vp, ctypes.c_uint64, vp, vp]
        lib.orc_ray_setup.restype = None
        lib.orc_half_to_double.argtypes = [ctypes.c_uint16]
        lib.orc_half_to_double.restype = ctypes.c_double
        _lib = lib
    return _lib


def _canvas_struct(cv):
    c = _Canvas()
    for k in range(3):
        c.origin[k] = cv.origin[k]
    c.root_edge = cv.root_edge
    c.R = cv.R
    c.max_depth = cv.max_depth
    c.leaf_format = cv.leaf_format
    c.nodes = cv.nodes.ctypes.data
    c.n_nodes = len(cv.nodes)
    c.leaves = cv.leaves.ctypes.data
    c.n_leaves = len(cv.leaves)
    return c


def _view_struct(v):
    s = _View()
    s.canvas = v["canvas_id"]
    s.W, s.H = v["W"], v["H"]
    for k in range(3):
        s.eye[k], s.right[k], s.up[k], s.fwd[k] = v["eye"][k], v["right"][k], v["up"][k], v["fwd"][k]
    s.tan_x, s.tan_y = v["tan_x"], v["tan_y"]
    s.out_offset_px = v["out_offset_px"]
    s.alpha_stop = v["alpha_stop"]
    return s


def ray_dir(view, x, y):
    d = np.zeros(3)
    _load().orc_ray_dir(ctypes.byref(_view_struct(view)), x, y, d.ctypes.data)
    return d


def ray_setup(canvas, view, px):
    """Unit directions (n, 3) and canvas chords t0, t1 (n each, root-edge units
    along d from the eye; 0, 0 for a miss) of pixels px (y*W + x) of a view:
    the oracle's own ray set-up."""
    px = np.ascontiguousarray(px, dtype=np.uint64)
    d = np.zeros((len(px), 3))
    t = np.zeros((len(px), 2))
    c = _canvas_struct(canvas)
    v = _view_struct(view)
    _load().orc_ray_setup(ctypes.byref(c), ctypes.byref(v), px.ctypes.data, len(px),
                          d.ctypes.data, t.ctypes.data)
    return d, t[:, 0], t[:, 1]


def half_to_double(h: int) -> float:
    return float(_load().orc_half_to_double(int(h)))


def render(canvases, views, ray_ids=None, eps_face=EPS_FACE, max_leaves=0, threads=None):
    """Trace rays with the oracle.

    ray_ids: uint64 array of (view << 32) | pixel, pixel = y*W + x; None means
    every pixel of every view in view order.  Returns a dict of per-ray arrays:
    rgba (n,4) f64, flags, n_leaves, alg_bytes, chord, sum_len and, when
    max_leaves > 0, the leaf node ids, local lengths and depths (n, max_leaves).
    """
    lib = _load()
    cs = (_Canvas * len(canvases))(*[_canvas_struct(c) for c in canvases])
    vs = (_View * len(views))(*[_view_struct(v) for v in views])
    if ray_ids is None:
        n = sum(v["W"] * v["H"] for v in views)
        ids_ptr = None
    else:
        ray_ids = np.ascontiguousarray(ray_ids, dtype=np.uint64)
        n = len(ray_ids)
        ids_ptr = ray_ids.ctypes.data
    out = dict(rgba=np.zeros((n, 4)), flags=np.zeros(n, np.uint32),
               n_leaves=np.zeros(n, np.uint32), alg_bytes=np.zeros(n), chord=np.zeros(n),
               sum_len=np.zeros(n))
    if max_leaves:
        out["leaf_ids"] = np.zeros((n, max_leaves), np.uint32)
        out["leaf_len"] = np.zeros((n, max_leaves))
        out["leaf_depth"] = np.zeros((n, max_leaves), np.uint8)
    p = lambda k: out[k].ctypes.data if k in out else None  # noqa: E731
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    rc = lib.orc_render(cs, len(canvases), vs, len(views), ids_ptr, n, eps_face, max_leaves,
                        p("rgba"), p("flags"), p("n_leaves"), p("alg_bytes"), p("chord"),
                        p("sum_len"), p("leaf_ids"), p("leaf_len"), p("leaf_depth"), int(threads))
    if rc != 0:
        raise RuntimeError("oracle render failed")
    out["threads"] = int(threads)
    return out

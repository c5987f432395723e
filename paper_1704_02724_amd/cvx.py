"""ctypes binding of libcvx (include/cvx.h): argument marshalling only.

Every function keeps the C name, converts Python/numpy arguments into the C
structures and raises ``CvxError`` on a non-zero status.  All compute runs in
the library's HIP kernels; there is no fallback: if ``lib/libcvx.so`` is
missing the import of this module fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

try:  # torch bundles a HIP runtime with the same soname as the system one; loading
    import torch  # noqa: F401  torch first makes libcvx bind to it, so torch's
except ImportError:  # streams and device pointers are valid inside libcvx
    torch = None

from .build import LIB_PATH

CVX_OK = 0
CVX_ERR_INVALID_ARG = -1
CVX_ERR_BAD_POOL = -2
CVX_ERR_OOM = -3
CVX_ERR_HIP = -4
CVX_ERR_NOT_FOUND = -5

CVX_LEAF_RGBA8_F16 = 0
CVX_LEAF_F64 = 1

CVX_VARIANT_FP32_REBASED = 0
CVX_VARIANT_FP64_PLAIN = 1
CVX_VARIANT_FP32_NAIVE = 2
CVX_VARIANT_FP32_CELL_LOCAL = 3
CVX_VARIANT_FP16_CELL_LOCAL = 4
VARIANTS = {"fp32_rebased": 0, "fp64_plain": 1, "fp32_naive": 2, "fp32_cell_local": 3,
            "fp16_cell_local": 4}

CVX_MAX_CANVASES = 64
CVX_MAX_DEPTH = 30
CVX_MAX_VIEWS = 4096
CVX_NOALLOC_MAX_VIEWS = 256

CVX_RAYFLAG_STEP_CAP = 1
CVX_RAYFLAG_FP64_EXIT = 2
CVX_RAYFLAG_BAD_LINK = 4

CVX_STAT_NAMES = ["rays", "leaves", "outer", "descent", "fp64_exit", "rebase", "steps", "slots"]
(CVX_STAT_RAYS, CVX_STAT_LEAVES, CVX_STAT_OUTER, CVX_STAT_DESCENT, CVX_STAT_FP64_EXIT,
 CVX_STAT_REBASE, CVX_STAT_STEPS, CVX_STAT_SLOTS) = range(8)
CVX_STAT_COUNT = 8

EXPORTED = ["cvx_create", "cvx_upload_pool", "cvx_render", "cvx_free_pool", "cvx_destroy",
            "cvx_last_error", "cvx_status_str", "cvx_validate_pool", "cvx_validate_views",
            "cvx_pool_bytes", "cvx_autotune", "cvx_edit_pool", "cvx_pool_nodes",
            "cvx_read_records", "cvx_read_payloads", "cvx_stroke_begin", "cvx_stroke_step",
            "cvx_render_noalloc"]

CVX_EDIT_PAINT = 0
CVX_EDIT_REFINE = 1
CVX_EDIT_COARSEN = 2
CVX_NONE_ID = 0xFFFFFFFF
CVX_MAX_STAMPS = 65536


class cvx_stroke(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_double * 3), ("sigma", ctypes.c_double),
                ("radius", ctypes.c_double), ("k_refine", ctypes.c_double),
                ("coarsen", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class cvx_canvas_desc(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("root_edge", ctypes.c_double),
                ("R", ctypes.c_uint32), ("max_depth", ctypes.c_uint32),
                ("leaf_format", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class cvx_view(ctypes.Structure):
    _fields_ = [("canvas_id", ctypes.c_int32), ("W", ctypes.c_uint32), ("H", ctypes.c_uint32),
                ("alpha_stop", ctypes.c_float), ("eye", ctypes.c_double * 3),
                ("right", ctypes.c_double * 3), ("up", ctypes.c_double * 3),
                ("fwd", ctypes.c_double * 3), ("tan_half_fov_x", ctypes.c_double),
                ("tan_half_fov_y", ctypes.c_double), ("out_offset_px", ctypes.c_uint64)]


class cvx_trace(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("ray_ids", ctypes.c_void_p),
                ("max_leaves", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("leaf_ids", ctypes.c_void_p), ("local_len", ctypes.c_void_p),
                ("local_len64", ctypes.c_void_p), ("n_leaves", ctypes.c_void_p),
                ("flags", ctypes.c_void_p), ("rgba", ctypes.c_void_p),
                ("end_point", ctypes.c_void_p)]


class cvx_render_opts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_uint32), ("tile_w", ctypes.c_uint32),
                ("tile_h", ctypes.c_uint32), ("workgroups", ctypes.c_uint32),
                ("wg_size", ctypes.c_uint32), ("use_graph", ctypes.c_uint32),
                ("out_f64", ctypes.c_uint32), ("top_lookup", ctypes.c_uint32),
                ("single_queue", ctypes.c_uint32), ("per_ray_start", ctypes.c_uint32),
                ("wide_offsets", ctypes.c_uint32), ("rays_per_wave", ctypes.c_uint32),
                ("refill_min", ctypes.c_uint32), ("chord_pieces", ctypes.c_uint32),
                ("cast_events", ctypes.c_void_p),
                ("trace", ctypes.POINTER(cvx_trace)), ("stats", ctypes.c_void_p)]


class cvx_edit(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("node", ctypes.c_uint32),
                ("first_payload", ctypes.c_uint64)]


# the same layout as a numpy record, for building long edit lists quickly
EDIT_DTYPE = np.dtype([("op", "<u4"), ("node", "<u4"), ("first_payload", "<u8")])
assert EDIT_DTYPE.itemsize == ctypes.sizeof(cvx_edit)


class cvx_tune_result(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_uint32), ("tile_h", ctypes.c_uint32),
                ("wg_size", ctypes.c_uint32), ("workgroups", ctypes.c_uint32),
                ("ms", ctypes.c_float), ("top_lookup", ctypes.c_uint32),
                ("single_queue", ctypes.c_uint32), ("rays_per_wave", ctypes.c_uint32),
                ("refill_min", ctypes.c_uint32), ("chord_pieces", ctypes.c_uint32)]


class CvxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{status_name(code)}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_lib.cvx_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, _vp]
_lib.cvx_upload_pool.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(cvx_canvas_desc), _vp,
                                 ctypes.c_uint64, _vp, ctypes.c_uint64]
_lib.cvx_render.argtypes = [_vp, _vp, ctypes.c_int, _vp, ctypes.POINTER(cvx_render_opts)]
_lib.cvx_render_noalloc.argtypes = [_vp, _vp, ctypes.c_int, _vp,
                                    ctypes.POINTER(cvx_render_opts)]
_lib.cvx_free_pool.argtypes = [_vp, ctypes.c_int]
_lib.cvx_destroy.argtypes = [_vp]
_lib.cvx_destroy.restype = None
_lib.cvx_last_error.argtypes = [_vp]
_lib.cvx_last_error.restype = ctypes.c_char_p
_lib.cvx_status_str.argtypes = [ctypes.c_int]
_lib.cvx_status_str.restype = ctypes.c_char_p
_lib.cvx_validate_pool.argtypes = [ctypes.POINTER(cvx_canvas_desc), _vp, ctypes.c_uint64, _vp,
                                   ctypes.c_uint64, ctypes.c_char_p, ctypes.c_size_t]
_lib.cvx_validate_views.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_int, ctypes.c_char_p,
                                    ctypes.c_size_t]
_lib.cvx_pool_bytes.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
_lib.cvx_edit_pool.argtypes = [_vp, ctypes.c_int, _vp, ctypes.c_uint32, _vp, ctypes.c_uint64, _vp]
_lib.cvx_pool_nodes.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
_lib.cvx_read_records.argtypes = [_vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, _vp]
_lib.cvx_read_payloads.argtypes = [_vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, _vp]
_lib.cvx_stroke_begin.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(cvx_stroke), _vp,
                                  ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]
_lib.cvx_stroke_step.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]
_lib.cvx_autotune.argtypes = [_vp, _vp, ctypes.c_int, _vp, ctypes.POINTER(cvx_render_opts),
                              ctypes.c_uint32, ctypes.POINTER(cvx_render_opts),
                              ctypes.POINTER(cvx_tune_result), ctypes.c_uint32,
                              ctypes.POINTER(ctypes.c_uint32)]


def library():
    return _lib


def status_name(code: int) -> str:
    return _lib.cvx_status_str(int(code)).decode()


cvx_status_str = status_name


def _check(ctx, rc):
    if rc != CVX_OK:
        msg = _lib.cvx_last_error(ctx).decode() if ctx else ""
        raise CvxError(rc, msg)


def make_desc(origin, root_edge, R, max_depth, leaf_format):
    d = cvx_canvas_desc()
    for k in range(3):
        d.origin[k] = float(origin[k])
    d.root_edge = float(root_edge)
    d.R, d.max_depth, d.leaf_format, d.reserved = int(R), int(max_depth), int(leaf_format), 0
    return d


def make_views(views):
    """List of view dicts -> ctypes array of cvx_view."""
    arr = (cvx_view * len(views))()
    for i, v in enumerate(views):
        a = arr[i]
        a.canvas_id, a.W, a.H = int(v["canvas_id"]), int(v["W"]), int(v["H"])
        a.alpha_stop = float(v["alpha_stop"])
        for k in range(3):
            a.eye[k], a.right[k], a.up[k], a.fwd[k] = (float(v["eye"][k]), float(v["right"][k]),
                                                       float(v["up"][k]), float(v["fwd"][k]))
        a.tan_half_fov_x, a.tan_half_fov_y = float(v["tan_x"]), float(v["tan_y"])
        a.out_offset_px = int(v["out_offset_px"])
    return arr


def cvx_create(device: int = 0, stream: int = 0):
    h = _vp()
    rc = _lib.cvx_create(ctypes.byref(h), int(device), _vp(int(stream)) if stream else None)
    if rc != CVX_OK:
        raise CvxError(rc, "cvx_create failed")
    return h


def cvx_upload_pool(ctx, canvas_id, desc, nodes, leaves):
    nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
    leaves = np.ascontiguousarray(leaves)
    _check(ctx, _lib.cvx_upload_pool(ctx, int(canvas_id), ctypes.byref(desc), nodes.ctypes.data,
                                     nodes.size // 2, leaves.ctypes.data if leaves.size else None,
                                     len(leaves)))


def cvx_render(ctx, views, out_ptr, opts=None):
    """views: ctypes array from make_views; out_ptr: device pointer (int)."""
    o = opts if opts is not None else cvx_render_opts()
    _check(ctx, _lib.cvx_render(ctx, ctypes.cast(views, _vp), len(views), _vp(int(out_ptr)),
                                ctypes.byref(o)))


def cvx_render_noalloc(ctx, views, out_ptr, opts=None):
    """The allocation-free render: same arguments and result as cvx_render,
    at most CVX_NOALLOC_MAX_VIEWS views, no graph."""
    o = opts if opts is not None else cvx_render_opts()
    _check(ctx, _lib.cvx_render_noalloc(ctx, ctypes.cast(views, _vp), len(views),
                                        _vp(int(out_ptr)), ctypes.byref(o)))


def cvx_autotune(ctx, views, out_ptr, base=None, reps=3, max_results=256):
    """Returns (best cvx_render_opts, list of (tile_w, tile_h, wg_size, workgroups, ms,
    top_lookup, single_queue, rays_per_wave, refill_min, chord_pieces))."""
    b = base if base is not None else cvx_render_opts()
    best = cvx_render_opts()
    res = (cvx_tune_result * max_results)()
    n = ctypes.c_uint32()
    _check(ctx, _lib.cvx_autotune(ctx, ctypes.cast(views, _vp), len(views), _vp(int(out_ptr)),
                                  ctypes.byref(b), int(reps), ctypes.byref(best), res,
                                  int(max_results), ctypes.byref(n)))
    rows = [(r.tile_w, r.tile_h, r.wg_size, r.workgroups, float(r.ms), r.top_lookup,
             r.single_queue, r.rays_per_wave, r.refill_min, r.chord_pieces)
            for r in res[:min(n.value, max_results)]]
    return best, rows


def cvx_edit_pool(ctx, canvas_id, edits, payloads):
    """edits: sequence of (op, node, first_payload) or an EDIT_DTYPE array;
    payloads: leaf records in the pool's format (numpy structured array).
    Returns the first child id per edit (CVX_NONE_ID for edits that are not
    REFINE)."""
    n = len(edits)
    if isinstance(edits, np.ndarray) and edits.dtype == EDIT_DTYPE:
        arr = np.ascontiguousarray(edits)
    elif n:
        arr = np.array([(int(a), int(b), int(c)) for a, b, c in edits], EDIT_DTYPE)
    else:
        arr = np.zeros(1, EDIT_DTYPE)
    payloads = np.ascontiguousarray(payloads)
    out = np.full(max(n, 1), CVX_NONE_ID, np.uint32)
    _check(ctx, _lib.cvx_edit_pool(ctx, int(canvas_id), arr.ctypes.data, n,
                                   payloads.ctypes.data if len(payloads) else None, len(payloads),
                                   out.ctypes.data))
    return out[:n]


def cvx_pool_nodes(ctx, canvas_id) -> int:
    b = ctypes.c_uint64()
    _check(ctx, _lib.cvx_pool_nodes(ctx, int(canvas_id), ctypes.byref(b)))
    return int(b.value)


def cvx_read_records(ctx, canvas_id, first=0, count=None):
    """Device node records as an (count, 4) uint32 array (diagnostic)."""
    if count is None:
        count = cvx_pool_nodes(ctx, canvas_id) - first
    out = np.zeros((count, 4), np.uint32)
    _check(ctx, _lib.cvx_read_records(ctx, int(canvas_id), int(first), int(count),
                                      out.ctypes.data if count else None))
    return out


def cvx_read_payloads(ctx, canvas_id, dtype, first=0, count=None):
    """Device leaf payloads indexed by node id, as an array of the pool's leaf
    dtype (diagnostic; entries of non-leaf ids are unspecified)."""
    if count is None:
        count = cvx_pool_nodes(ctx, canvas_id) - first
    out = np.zeros(count, dtype)
    _check(ctx, _lib.cvx_read_payloads(ctx, int(canvas_id), int(first), int(count),
                                       out.ctypes.data if count else None))
    return out


def cvx_stroke_begin(ctx, canvas_id, stamps, rgb, sigma, radius, k_refine, coarsen=False) -> int:
    """Start a brush stroke (stamps: (n, 4) x, y, z, r in world units); returns
    the number of leaves waiting for a split (or, for a coarsening stroke with
    no split to make, of cells waiting for a merge)."""
    st = cvx_stroke()
    st.rgb[:] = [float(v) for v in rgb]
    st.sigma, st.radius, st.k_refine = float(sigma), float(radius), float(k_refine)
    st.coarsen = 1 if coarsen else 0
    arr = np.ascontiguousarray(stamps, np.float64).reshape(-1, 4)
    pend = ctypes.c_uint64()
    _check(ctx, _lib.cvx_stroke_begin(ctx, int(canvas_id), ctypes.byref(st),
                                      arr.ctypes.data if len(arr) else None, len(arr),
                                      ctypes.byref(pend)))
    return int(pend.value)


def cvx_stroke_step(ctx, canvas_id) -> int:
    """One deferred level of the stroke in progress; returns the leaves still
    waiting for a split (0: the stroke is complete)."""
    pend = ctypes.c_uint64()
    _check(ctx, _lib.cvx_stroke_step(ctx, int(canvas_id), ctypes.byref(pend)))
    return int(pend.value)


def cvx_free_pool(ctx, canvas_id):
    _check(ctx, _lib.cvx_free_pool(ctx, int(canvas_id)))


def cvx_destroy(ctx):
    _lib.cvx_destroy(ctx)


def cvx_last_error(ctx) -> str:
    return _lib.cvx_last_error(ctx).decode()


def cvx_pool_bytes(ctx, canvas_id) -> int:
    b = ctypes.c_uint64()
    _check(ctx, _lib.cvx_pool_bytes(ctx, int(canvas_id), ctypes.byref(b)))
    return int(b.value)


def cvx_validate_pool(desc, nodes, leaves):
    """Host-only validation; returns (status, message)."""
    nodes = np.ascontiguousarray(nodes, dtype=np.uint32)
    leaves = np.ascontiguousarray(leaves)
    buf = ctypes.create_string_buffer(512)
    rc = _lib.cvx_validate_pool(ctypes.byref(desc), nodes.ctypes.data, nodes.size // 2,
                                leaves.ctypes.data if leaves.size else None, len(leaves), buf, 512)
    return rc, buf.value.decode()


def cvx_validate_views(views, descs):
    """Host-only view validation against a list of canvas descs (None = absent)."""
    ptrs = (ctypes.POINTER(cvx_canvas_desc) * len(descs))(
        *[ctypes.pointer(d) if d is not None else ctypes.POINTER(cvx_canvas_desc)() for d in descs])
    buf = ctypes.create_string_buffer(512)
    rc = _lib.cvx_validate_views(ctypes.cast(views, _vp), len(views), ctypes.cast(ptrs, _vp),
                                 len(descs), buf, 512)
    return rc, buf.value.decode()


def make_opts(variant="fp32_rebased", tile=(0, 0), workgroups=0, wg_size=0, use_graph=False,
              out_f64=False, trace=None, stats_ptr=0, top_lookup=0, single_queue=0,
              per_ray_start=0, wide_offsets=0, rays_per_wave=0, refill_min=0,
              chord_pieces=0, cast_events=0):
    o = cvx_render_opts()
    o.cast_events = _vp(int(cast_events)) if cast_events else None
    o.chord_pieces = int(chord_pieces)
    o.wide_offsets = int(wide_offsets)
    o.rays_per_wave = int(rays_per_wave)
    o.refill_min = int(refill_min)
    o.top_lookup = int(top_lookup)
    o.single_queue = int(single_queue)
    o.per_ray_start = int(per_ray_start)
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.tile_w, o.tile_h = int(tile[0]), int(tile[1])
    o.workgroups, o.wg_size = int(workgroups), int(wg_size)
    o.use_graph, o.out_f64 = int(bool(use_graph)), int(bool(out_f64))
    if trace is not None:
        o.trace = ctypes.pointer(trace)
    o.stats = _vp(int(stats_ptr)) if stats_ptr else None
    return o

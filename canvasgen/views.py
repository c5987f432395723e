"""Seeded pinhole views (input generation only).

A view is a pinhole camera in canvas (world) coordinates: an FP64 eye
position, an orthonormal basis (right, up, fwd), the tangents of the half
fields of view, an image size, the canvas it looks at and where its pixels go
in the output buffer.  Keeping the eye in FP64 stands in for the end of the
chain of canvas->VR->HMD->eye transforms the paper keeps precise (Sec. 6.1).
"""
from __future__ import annotations

import numpy as np


def make_view(eye, fwd, tan_x, W, H, canvas_id=0, up_hint=(0.0, 1.0, 0.0), out_offset_px=0,
              alpha_stop=1.0, tan_y=None):
    f = np.asarray(fwd, np.float64)
    f = f / np.linalg.norm(f)
    u0 = np.asarray(up_hint, np.float64)
    if abs(float(np.dot(u0, f))) > 0.9:
        u0 = np.array([1.0, 0.0, 0.0]) if abs(f[0]) < 0.9 else np.array([0.0, 0.0, 1.0])
    right = np.cross(f, u0)
    right /= np.linalg.norm(right)
    up = np.cross(right, f)
    up /= np.linalg.norm(up)
    if tan_y is None:
        tan_y = float(tan_x) * H / W
    return dict(canvas_id=int(canvas_id), eye=tuple(float(v) for v in eye),
                right=tuple(right.tolist()), up=tuple(up.tolist()), fwd=tuple(f.tolist()),
                tan_x=float(tan_x), tan_y=float(tan_y), W=int(W), H=int(H),
                out_offset_px=int(out_offset_px), alpha_stop=float(alpha_stop))


def stereo_pair(eye, fwd, ipd, tan_x, W, H, canvas_id=0, out_offset_px=0, alpha_stop=1.0):
    """Two parallel views whose eyes sit ipd apart along the shared right axis."""
    c = make_view(eye, fwd, tan_x, W, H, canvas_id, alpha_stop=alpha_stop)
    r = np.asarray(c["right"])
    e = np.asarray(eye, np.float64)
    left = make_view(e - 0.5 * ipd * r, fwd, tan_x, W, H, canvas_id, out_offset_px=out_offset_px,
                     alpha_stop=alpha_stop)
    right = make_view(e + 0.5 * ipd * r, fwd, tan_x, W, H, canvas_id,
                      out_offset_px=out_offset_px + W * H, alpha_stop=alpha_stop)
    return [left, right]


def eye_near_stroke(rng: np.random.Generator, strokes, r_max=2.0 ** -16):
    """Place an eye just outside a small painted stroke, looking at one of its stamps.

    Pick a stroke with radius <= r_max (the smallest one if none qualifies),
    start at one of its stamp centres and walk along a random direction in
    steps of r/2 until the point is at least 2r outside every stamp of that
    stroke (and still inside the unit canvas).  Returns (eye, fwd, r).
    """
    ok = np.nonzero(strokes.radius <= r_max)[0]
    if len(ok) == 0:
        ok = np.array([int(np.argmin(strokes.radius))])
    for _ in range(1000):
        s = int(ok[rng.integers(len(ok))])
        st = strokes.stamps_of(s)
        if len(st) == 0:
            continue
        c = st[rng.integers(len(st)), :3]
        r = float(strokes.radius[s])
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        p = c.copy()
        for m in range(1, 100000):
            p = c + m * 0.5 * r * u
            if np.min(np.linalg.norm(st[:, :3] - p[None, :], axis=1)) >= 3.0 * r:
                break
        if np.all(p > 0.0) and np.all(p < 1.0):
            return p, c - p, r
    raise RuntimeError("could not place an eye inside the canvas")

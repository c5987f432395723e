"""The workloads: seeded stroke canvases and their views.

Each workload fixes the stroke recipe, the tree limits (max depth D, refine
factor k: a cell overlapping a stamp is split while its edge exceeds r/k), the
leaf format and the cameras.  Every random number comes from one
``Generator(PCG64(seed))`` per workload, drawn in the order: strokes, then
cameras.

  tiny      R=1, D=12, 16 strokes r in 2^[-8,-4], k=4; one 256x256 view, 60 deg
            horizontal FOV, eye (0.5,0.5,-0.5) looking +z.
  depth24   2,000 strokes r in 2^[-20,-3], D=24, k=4 (k=10 variant reaches 24);
            stereo pair 1920x1080 per eye, 90 deg FOV, eye just outside a stroke
            of radius <= 2^-16, interpupillary distance r/2.
  depth30   500 strokes r in 2^[-10,-3] plus 200 strokes r in 2^[-27,-25] whose
            start points lie in a 2^-22 box (corner uniform in [0.5,1)^3 snapped
            to 2^-22); D=30; one 1024x1024 view 2^-24 from the cluster centre
            whose image spans 2^-24 at that distance.
  batch     8 canvases with D = 16,18,19,21,23,25,26,28, stroke counts
            log-uniform in [200, 5000], r in 2^[-(D-2),-3], k=4; 64 views, view v
            on canvas v mod 8, pairs (2j, 2j+1) are stereo pairs with a square
            side uniform in [256, 2160].  Pair j looks at canvas j mod 8 (a
            stereo pair shares one canvas), so each canvas gets 4 pairs.
  large     55,000 strokes r in 2^[-24,-2], D=26, k=4 (about 1.5 G nodes: the
            pool grows by about 26.9 K nodes per stroke, so 100,000 strokes
            would pass the 2^31 node ids of the pool format); stereo
            2160x2160 per eye, rays stop once accumulated alpha reaches 0.99.
"""
from __future__ import annotations

import math

import numpy as np

from .pool import LEAF_F64, LEAF_RGBA8_F16, build_from_strokes
from .strokes import StrokeSet, gen_strokes
from .views import eye_near_stroke, make_view, stereo_pair


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


class Workload:
    def __init__(self, name, canvases, views, strokes=None, meta=None):
        self.name = name
        self.canvases = canvases      # list of Canvas
        self.views = views            # list of view dicts
        self.strokes = strokes or []  # list of StrokeSet (one per canvas)
        self.meta = dict(meta or {})

    @property
    def n_rays(self):
        return sum(v["W"] * v["H"] for v in self.views)

    @property
    def out_pixels(self):
        return max(v["out_offset_px"] + v["W"] * v["H"] for v in self.views)


def tiny(seed=1, leaf_format=LEAF_F64, k=4.0, W=256, H=256, R=1):
    rng = _rng(seed)
    st = gen_strokes(rng, 16, -8.0, -4.0)
    cv = build_from_strokes(st, R, 12, k, leaf_format)
    v = make_view((0.5, 0.5, -0.5), (0.0, 0.0, 1.0), math.tan(math.radians(30.0)), W, H)
    return Workload("tiny", [cv], [v], [st], dict(seed=seed, k=k, D=12))


def depth24(seed=24, k=4.0, W=1920, H=1080, leaf_format=LEAF_RGBA8_F16, threads=0):
    rng = _rng(seed)
    st = gen_strokes(rng, 2000, -20.0, -3.0)
    cv = build_from_strokes(st, 1, 24, k, leaf_format, split_depth=5, threads=threads)
    eye, fwd, r = eye_near_stroke(rng, st, 2.0 ** -16)
    views = stereo_pair(eye, fwd, 0.5 * r, 1.0, W, H)
    return Workload("depth24", [cv], views, [st], dict(seed=seed, k=k, D=24, eye_stroke_r=r))


def depth30(seed=30, k=4.0, W=1024, H=1024, leaf_format=LEAF_RGBA8_F16, threads=0):
    rng = _rng(seed)
    coarse = gen_strokes(rng, 500, -10.0, -3.0)
    box = 2.0 ** -22
    corner = np.floor(rng.uniform(0.5, 1.0, 3) / box) * box
    fine = gen_strokes(rng, 200, -27.0, -25.0, box_lo=corner, box_size=box)
    st = StrokeSet.concat([coarse, fine])
    cv = build_from_strokes(st, 1, 30, k, leaf_format, split_depth=5, threads=threads)
    centre = corner + 0.5 * box
    u = rng.normal(size=3)
    u /= np.linalg.norm(u)
    dist = 2.0 ** -24
    eye = centre - dist * u
    v = make_view(eye, u, 0.5, W, H)  # image spans 2*0.5*dist = 2^-24 at the centre
    return Workload("depth30", [cv], [v], [st], dict(seed=seed, k=k, D=30, corner=corner.tolist()))


BATCH_DEPTHS = (16, 18, 19, 21, 23, 25, 26, 28)


def batch(seed=4000, leaf_format=LEAF_RGBA8_F16, threads=0, side_scale=1.0):
    canvases, strokes, views = [], [], []
    for ci, D in enumerate(BATCH_DEPTHS):
        rng = _rng(seed + ci + 1)
        n = int(round(math.exp(rng.uniform(math.log(200), math.log(5000)))))
        st = gen_strokes(rng, n, -(D - 2.0), -3.0)
        canvases.append(build_from_strokes(st, 1, D, 4.0, leaf_format, split_depth=5,
                                           threads=threads))
        strokes.append(st)
    rng = _rng(seed)
    off = 0
    for j in range(32):
        ci = j % 8
        side = int(rng.integers(256, 2161))
        side = max(8, int(side * side_scale))
        eye, fwd, r = eye_near_stroke(rng, strokes[ci], 2.0 ** -16)
        pair = stereo_pair(eye, fwd, 0.5 * r, 1.0, side, side, canvas_id=ci, out_offset_px=off)
        off += 2 * side * side
        views.extend(pair)
    return Workload("batch", canvases, views, strokes, dict(seed=seed, depths=BATCH_DEPTHS))


LARGE_STROKES = 55000


def large(seed=5, leaf_format=LEAF_RGBA8_F16, threads=0, W=2160, H=2160,
          n_strokes=LARGE_STROKES):
    rng = _rng(seed)
    st = gen_strokes(rng, n_strokes, -24.0, -2.0)
    cv = build_from_strokes(st, 1, 26, 4.0, leaf_format, split_depth=5, threads=threads,
                            verbose=n_strokes >= 10000)
    eye, fwd, r = eye_near_stroke(rng, st, 2.0 ** -16)
    views = stereo_pair(eye, fwd, 0.5 * r, 1.0, W, H, alpha_stop=0.99)
    return Workload("large", [cv], views, [st], dict(seed=seed, D=26))

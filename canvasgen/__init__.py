"""Seeded input generation for the deep-octree ray caster.

Holds the stroke recipe, the host tree builder that turns strokes into the
node pool, small hand-shaped trees and the cameras.  It contains none of the
ray traversal or compositing arithmetic: both the CPU oracle and the GPU path
consume what it produces.
"""
from .pool import (LEAF, LEAF_DTYPE, LEAF_F64, LEAF_RGBA8_F16, NONE, Canvas, build_from_strokes,
                   build_lib)
from .strokes import StrokeSet, gen_strokes
from .views import eye_near_stroke, make_view, stereo_pair

__all__ = ["LEAF", "LEAF_DTYPE", "LEAF_F64", "LEAF_RGBA8_F16", "NONE", "Canvas",
           "build_from_strokes", "build_lib", "StrokeSet", "gen_strokes", "eye_near_stroke",
           "make_view", "stereo_pair"]

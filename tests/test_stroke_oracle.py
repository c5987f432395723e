"""CPU pins of the stroke oracle (oracle/stroke.py).

* Against the canvas builder, an independent implementation of the same
  painting rules that applies strokes in sequence: painting stroke n into the
  builder's canvas of strokes 1..n-1 gives exactly (FP64 leaves) the builder's
  canvas of strokes 1..n, for several seeds, root arrays and depths.
* Brute-force properties: after a stroke every leaf the stamps overlap is at
  the brush resolution or the max depth; every leaf they miss is unchanged;
  the leaves still tile the canvas.
* The RGBA8 + half-kappa path equals the FP64 path encoded, on a canvas whose
  payloads both formats hold exactly (every leaf the stroke changes; the rest
  are untouched in both).
* The deferred passes (immediate paint, then one level of splits at a time)
  end on the result of the stroke applied at once.
* The lossless coarsening: a uniform canvas under a stroke that covers it
  collapses to its roots with the optical depth doubled per level; on
  stroked canvases it leaves no mergeable cell and the FP64 oracle renders
  the coarsened canvas like the uncoarsened one.
"""
import math

import numpy as np
import pytest

from canvasgen import LEAF_F64, LEAF_RGBA8_F16, trees
from canvasgen.pool import build_from_strokes
from canvasgen.strokes import StrokeSet, gen_strokes
from oracle import stroke as so


def _subset(st, n):
    return StrokeSet(st.radius[:n], st.rgb[:n], st.sigma[:n], st.stamp_off[:n + 1],
                     st.stamps[:st.stamp_off[n]])


def _canon(cv):
    return so.canonical_from_pool(cv.nodes, cv.leaves, cv.R)


def _apply(cv, st, i, k, leaves=None, fmt=None):
    return so.apply_stroke(_canon(cv) if leaves is None else leaves,
                           cv.leaf_format if fmt is None else fmt, cv.R, cv.max_depth,
                           cv.root_edge, cv.origin, st.stamps_of(i), st.rgb[i], st.sigma[i],
                           st.radius[i], k)


@pytest.mark.parametrize("R,D,n,lg,seed", [(1, 8, 6, (-6, -3), 1), (2, 7, 5, (-6, -3), 2),
                                          (1, 10, 4, (-9, -5), 3), (3, 6, 8, (-5, -2), 4)])
def test_stroke_matches_sequential_builder(R, D, n, lg, seed):
    k = 4.0
    st = gen_strokes(np.random.Generator(np.random.PCG64(seed)), n, *lg)
    prev = build_from_strokes(_subset(st, n - 1), R, D, k, LEAF_F64)
    full = build_from_strokes(st, R, D, k, LEAF_F64)
    got, split = _apply(prev, st, n - 1, k)
    want = _canon(full)
    assert set(got) == set(want)
    bad = [c for c in want if got[c] != want[c]]
    assert not bad, (len(bad), bad[:3])
    # the last stroke changed something and split something
    before = _canon(prev)
    assert split and any(before.get(c) != v for c, v in want.items())


def test_stroke_properties_brute_force():
    rng = np.random.Generator(np.random.PCG64(11))
    cv = trees.random_tree(2, 6, seed=11, max_nodes=4000, leaf_format=LEAF_F64)
    before = _canon(cv)
    st = gen_strokes(rng, 3, -5, -3)
    k = 4.0
    for i in range(st.n):
        after, _ = _apply(cv, st, i, k, leaves=before)
        stamps = st.stamps_of(i)
        hmin = st.radius[i] / k
        vol = 0.0
        for (d, x, y, z), pay in after.items():
            e = math.ldexp(cv.root_edge, -d)
            lo = np.array([x, y, z], np.float64) * e
            near = np.maximum(np.maximum(lo[None, :] - stamps[:, :3], 0.0),
                              stamps[:, :3] - (lo[None, :] + e))
            overlap = np.any((near * near).sum(1) < stamps[:, 3] ** 2)
            if overlap:
                assert e <= hmin or d == cv.max_depth
            vol += 8.0 ** -d
        assert vol == pytest.approx(cv.R ** 3)
        for cell, pay in before.items():
            d, x, y, z = cell
            e = math.ldexp(cv.root_edge, -d)
            lo = np.array([x, y, z], np.float64) * e
            near = np.maximum(np.maximum(lo[None, :] - stamps[:, :3], 0.0),
                              stamps[:, :3] - (lo[None, :] + e))
            if not np.any((near * near).sum(1) < stamps[:, 3] ** 2):
                assert after[cell] == pay
        before = after


def test_rgba8_path_is_the_f64_path_encoded():
    cv8 = trees.random_tree(1, 6, seed=12, max_nodes=3000, leaf_format=LEAF_RGBA8_F16,
                            kappa_range=(0.0, 4.0))
    leaves8 = _canon(cv8)
    leaves64 = {c: so.decode(p, so.RGBA8_F16) for c, p in leaves8.items()}
    st = gen_strokes(np.random.Generator(np.random.PCG64(12)), 4, -5, -3)
    for i in range(st.n):
        a8, s8 = _apply(cv8, st, i, 4.0, leaves=leaves8, fmt=so.RGBA8_F16)
        a64, s64 = _apply(cv8, st, i, 4.0, leaves=leaves64, fmt=so.F64)
        assert s8 == s64 and set(a8) == set(a64)
        for c in a8:
            if leaves8.get(c) == a8[c]:          # untouched (its A byte is the generator's)
                assert a64[c] == leaves64[c], c
            else:
                assert a8[c] == so.encode(a64[c], so.RGBA8_F16), c
        leaves8 = a8
        leaves64 = {c: so.decode(p, so.RGBA8_F16) for c, p in a8.items()}


@pytest.mark.parametrize("fmt", [LEAF_F64, LEAF_RGBA8_F16])
def test_deferred_passes_end_on_the_stroke_at_once(fmt):
    """Immediate paint of the existing leaves, then one level of splits per
    pass whose children start from the payload before the stroke."""
    cv = trees.random_tree(1, 7, seed=13, max_nodes=2000, leaf_format=fmt)
    st = gen_strokes(np.random.Generator(np.random.PCG64(13)), 2, -7, -4)
    k = 4.0
    for i in range(st.n):
        start = _canon(cv)
        want, _ = _apply(cv, st, i, k, leaves=start)
        args = (cv.R, cv.max_depth, cv.root_edge, cv.origin, st.stamps_of(i), st.rgb[i],
                st.sigma[i], st.radius[i], k)
        cur, pending = so.immediate(start, fmt, *args)
        pre = {c: start[c] for c in pending}
        passes = 0
        while pending:
            passes += 1
            kids = {}
            for (d, x, y, z) in pending:
                del cur[(d, x, y, z)]
                cp = so.child_payload(pre[(d, x, y, z)], fmt)
                for o in range(8):
                    kids[(d + 1, 2 * x + (o & 1), 2 * y + ((o >> 1) & 1),
                          2 * z + ((o >> 2) & 1))] = cp
            painted, pending = so.immediate(kids, fmt, *args)
            pre = {c: kids[c] for c in pending}
            cur.update(painted)
        assert 0 < passes <= cv.max_depth
        assert cur == want


def _pool_from(leaves, R, max_depth, fmt):
    """A host pool of a canonical dict (F64 leaves), for the render oracle."""
    cells = set(leaves)
    inner = {(d - k, x >> k, y >> k, z >> k) for (d, x, y, z) in cells for k in range(1, d + 1)}
    return trees.from_refinement(R, max_depth, lambda d, c: (d, *c) in inner,
                                 lambda d, c: leaves[(d, *c)], fmt)


def test_merge_collapses_a_uniform_canvas():
    cv = trees.from_refinement(2, 4, lambda d, c: d < 3, lambda d, c: (0.25, 0.5, 0.75, 0.125),
                               LEAF_F64)
    leaves = _canon(cv)
    big = np.array([[0.5, 0.5, 0.5, 2.0]])            # covers the whole canvas
    out, merged = so.merge_uniform(leaves, so.F64, cv.root_edge, cv.origin, big)
    assert set(out) == {(0, x, y, z) for x in range(2) for y in range(2) for z in range(2)}
    assert all(p == (0.25, 0.5, 0.75, 0.125 * 8) for p in out.values())
    assert len(merged) == 8 * (1 + 8 + 64)             # depth 2, 1 and 0 cells


@pytest.mark.parametrize("fmt", [LEAF_F64, LEAF_RGBA8_F16])
def test_merge_after_strokes_is_lossless_and_complete(fmt):
    from oracle import oracle
    cv = trees.from_refinement(1, 8, lambda d, c: d < 2, lambda d, c: (0.3, 0.6, 0.2, 0.5), fmt)
    st = gen_strokes(np.random.Generator(np.random.PCG64(14)), 2, -4, -3)
    k = 4.0
    leaves = _canon(cv)
    for i in range(st.n):
        args = (cv.R, cv.max_depth, cv.root_edge, cv.origin, st.stamps_of(i), st.rgb[i],
                st.sigma[i], st.radius[i], k)
        painted, _ = so.apply_stroke(leaves, fmt, *args)
        merged, cells = so.merge_uniform(painted, fmt, cv.root_edge, cv.origin, st.stamps_of(i))
        assert cells and len(merged) < len(painted)
        # no mergeable cell left under the stroke
        again, more = so.merge_uniform(merged, fmt, cv.root_edge, cv.origin, st.stamps_of(i))
        assert not more and again == merged
        if fmt == LEAF_F64:
            # the render oracle sees the same canvas
            rng = np.random.Generator(np.random.PCG64(15 + i))
            from helpers import random_rays, ray_views
            vs = ray_views(*random_rays(rng, 300))
            a = oracle.render([_pool_from(painted, 1, cv.max_depth, fmt)], vs)
            b = oracle.render([_pool_from(merged, 1, cv.max_depth, fmt)], vs)
            np.testing.assert_allclose(b["rgba"], a["rgba"], atol=1e-12)
            assert b["n_leaves"].sum() < a["n_leaves"].sum()
        leaves = merged


def test_exact_boundaries_of_the_rules():
    """Exact dyadic cases of the inequalities of the rules (Sec. 5.1-5.2 read
    as in the builder): a leaf is split only while its edge exceeds radius /
    k, so a brush of radius 2^-4 with k = 4 stops at edge 2^-6 = radius / k;
    a stamp reaches a leaf only when the leaf's box lies at a distance below
    its radius, so a sphere that only touches a box (distance equal to the
    radius, exact in FP64) leaves that leaf alone; and a leaf whose centre
    lies on a stamp's sphere takes the stroke."""
    cv = trees.from_refinement(1, 10, lambda d, c: d < 1, lambda d, c: (0.2, 0.4, 0.6, 1.0),
                               LEAF_F64)
    leaves = _canon(cv)
    r = 2.0 ** -4
    # touches the box of leaf (1, 0, 0, 0) = [0, 0.5]^3 from x = 0.75, inside leaf (1, 1, 0, 0)
    stamp = np.array([[0.75, 0.25, 0.25, 0.25]])
    out, split = so.apply_stroke(leaves, so.F64, 1, 10, 1.0, (0.0, 0.0, 0.0), stamp,
                                 (1.0, 0.0, 0.0), 10.0, 0.25, 4.0)
    assert out[(1, 0, 0, 0)] == leaves[(1, 0, 0, 0)] and (1, 0, 0, 0) not in split
    assert (1, 1, 0, 0) in split
    # a brush of radius 2^-4, one stamp inside leaf (1, 1, 1, 1)
    stamp = np.array([[0.7, 0.7, 0.7, r]])
    out, split = so.apply_stroke(leaves, so.F64, 1, 10, 1.0, (0.0, 0.0, 0.0), stamp,
                                 (1.0, 0.0, 0.0), 10.0, r, 4.0)
    assert max(d for (d, _, _, _) in out) == 6
    assert max(d for (d, _, _, _) in split) == 5
    # a leaf takes the stroke when its centre lies in a stamp, the sphere's
    # surface included: on a canvas that cannot refine further, a stamp of
    # radius 0.5 at distance exactly 0.5 from the centre of leaf (1, 0, 0, 0)
    flat = trees.from_refinement(1, 1, lambda d, c: d < 1, lambda d, c: (0.2, 0.4, 0.6, 1.0),
                                 LEAF_F64)
    fl = _canon(flat)
    stamp = np.array([[0.75, 0.25, 0.25, 0.5]])
    out, split = so.apply_stroke(fl, so.F64, 1, 1, 1.0, (0.0, 0.0, 0.0), stamp,
                                 (1.0, 0.0, 0.0), 10.0, 0.5, 4.0)
    assert not split
    assert out[(1, 0, 0, 0)] != fl[(1, 0, 0, 0)]      # centre on the sphere: painted
    assert out[(1, 0, 1, 0)] == fl[(1, 0, 1, 0)]      # overlapped, centre outside

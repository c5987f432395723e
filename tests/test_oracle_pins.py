"""Pins for the CPU FP64 oracle: brute force, closed forms, invariants.

Each check fixes the oracle to something other than itself: per-leaf slab
intersection of every leaf (brute force), exact rational 3D-DDA walks on
uniform lattices (Amanatides & Woo), the closed-form transmittance of a single
homogeneous cell, the analytic front-to-back result of two cells, refinement
invariance of a homogeneous region, and the chord invariant sum(l*h) = t1-t0.
"""
from fractions import Fraction as F
import math

import numpy as np
import pytest

from canvasgen import LEAF_F64, LEAF_RGBA8_F16, make_view
from canvasgen import trees
from oracle import oracle

from bruteforce import leaf_boxes, sequence
from helpers import random_rays, ray_views

def test_half_decode_matches_ieee():
    bits = np.arange(65536, dtype=np.uint16)
    ref = bits.view(np.float16).astype(np.float64)
    ok = np.isfinite(ref)
    got = np.array([oracle.half_to_double(int(b)) for b in bits[ok][::7]])
    np.testing.assert_array_equal(got, ref[ok][::7])


def test_ray_directions_pinhole_geometry():
    W, H = 64, 32
    v = make_view((0.1, 0.2, 0.3), (0.3, -0.2, 0.9), 1.0, W, H)
    R_, U_, F_ = (np.asarray(v[k]) for k in ("right", "up", "fwd"))
    tan = np.zeros((H, W, 2))
    for y in range(H):
        for x in range(W):
            d = oracle.ray_dir(v, x, y)
            assert abs(np.linalg.norm(d) - 1.0) < 1e-15
            tan[y, x] = (d @ R_ / (d @ F_), d @ U_ / (d @ F_))
    # left/right and top/bottom mirror symmetry; row 0 is the top row
    np.testing.assert_allclose(tan[:, ::-1, 0], -tan[:, :, 0], atol=1e-14)
    np.testing.assert_allclose(tan[::-1, :, 1], -tan[:, :, 1], atol=1e-14)
    assert np.all(tan[0, :, 1] > 0) and np.all(tan[:, 0, 0] < 0)
    # a pinhole samples the image plane uniformly
    dx = np.diff(tan[:, :, 0], axis=1)
    np.testing.assert_allclose(dx, dx[0, 0], rtol=1e-12)
    # the outermost pixel centres sit half a pixel inside the field of view
    assert abs(tan[0, -1, 0] - (1.0 - 1.0 / W)) < 1e-12
    assert abs(tan[0, 0, 1] - (0.5 - 0.5 / H)) < 1e-12


@pytest.mark.parametrize("fmt", [LEAF_F64, LEAF_RGBA8_F16])
def test_single_homogeneous_cell_closed_form(fmt):
    col, kap = (60 / 255.0, 120 / 255.0, 240 / 255.0), 0.75
    cv = trees.single_cell(col, kap, fmt)
    rng = np.random.Generator(np.random.PCG64(3))
    eyes, dirs, lens = [], [], []
    for i in range(40):
        y, z = rng.uniform(0.05, 0.95, 2)
        ax = i % 3
        sgn = 1.0 if i % 2 == 0 else -1.0
        if i % 4 < 2:  # from outside: the chord is the whole edge
            e = np.roll(np.array([(-0.5 if sgn > 0 else 1.5), y, z]), ax)
            L = 1.0
        else:          # eye inside: the chord is the distance to the far face
            x0 = rng.uniform(0.1, 0.9)
            e = np.roll(np.array([x0, y, z]), ax)
            L = (1.0 - x0) if sgn > 0 else x0
        d = np.roll(np.array([sgn, 0.0, 0.0]), ax)
        eyes.append(e)
        dirs.append(d)
        lens.append(L)
    out = oracle.render([cv], ray_views(eyes, dirs))
    A = 1.0 - np.exp(-kap * np.asarray(lens))
    assert np.all(out["flags"] == 0)
    np.testing.assert_allclose(out["rgba"][:, 3], A, rtol=0, atol=1e-14)
    for ch in range(3):
        np.testing.assert_allclose(out["rgba"][:, ch], col[ch] * A, rtol=0, atol=1e-14)
    assert np.all(out["n_leaves"] == 1)


def test_two_cells_front_to_back_order():
    # R = 2 root array (Sec. 4): roots (0,0,0) and (1,0,0) hold different media
    pay = {(0, 0, 0): (1.0, 0.0, 0.0, 0.4), (1, 0, 0): (0.0, 0.0, 1.0, 1.7)}
    cv = trees.from_refinement(2, 0, lambda d, c: False,
                               lambda d, c: pay.get(tuple(c), (0.0, 1.0, 0.0, 0.0)), LEAF_F64)
    e1, e2 = math.exp(-0.4), math.exp(-1.7)   # each root is crossed over one root edge
    vs = ray_views([(-1.0, 0.2, 0.3), (2.0, 0.2, 0.3)], [(1.0, 0, 0), (-1.0, 0, 0)])
    out = oracle.render([cv], vs)
    red_first = np.array([(1 - e1), 0.0, e1 * (1 - e2), 1 - e1 * e2])
    blue_first = np.array([e2 * (1 - e1), 0.0, (1 - e2), 1 - e1 * e2])
    np.testing.assert_allclose(out["rgba"][0], red_first, atol=1e-15)
    np.testing.assert_allclose(out["rgba"][1], blue_first, atol=1e-15)


@pytest.mark.parametrize("depth", [1, 3, 5])
def test_refinement_invariance(depth):
    col, kap = (0.2, 0.5, 0.9), 2.0
    coarse = trees.single_cell(col, kap, LEAF_F64)
    fine = trees.from_refinement(1, depth, lambda d, c: True,
                                 lambda d, c: (*col, kap * 2.0 ** -d), LEAF_F64)
    rng = np.random.Generator(np.random.PCG64(10 + depth))
    eyes, dirs = random_rays(rng, 200)
    vs = ray_views(eyes, dirs)
    a = oracle.render([coarse], vs)
    b = oracle.render([fine], vs)
    np.testing.assert_allclose(b["rgba"], a["rgba"], atol=1e-12)
    hit = a["chord"] > 0
    assert hit.sum() > 150
    assert np.all(b["n_leaves"][hit] >= 1)


def _leaf_seq_mismatches(cv, vs, max_leaves=600):
    out = oracle.render([cv], vs, max_leaves=max_leaves)
    boxes = leaf_boxes(cv)
    n_checked = 0
    for i, v in enumerate(vs):
        if out["flags"][i] & oracle.FLAG_NEAR_FACE:
            continue
        d = oracle.ray_dir(v, 0, 0)
        ids, lens = sequence(cv, boxes, v["eye"], d)
        n = int(out["n_leaves"][i])
        assert n <= max_leaves
        assert n == len(ids), (i, n, len(ids))
        np.testing.assert_array_equal(out["leaf_ids"][i, :n], ids)
        np.testing.assert_allclose(out["leaf_len"][i, :n], lens, atol=1e-9)
        n_checked += 1
    return n_checked


@pytest.mark.parametrize("R,depth,seed", [(1, 4, 0), (1, 6, 1), (2, 5, 2), (3, 4, 3)])
def test_sequences_match_brute_force(R, depth, seed):
    cv = trees.random_tree(R, depth, seed=seed, p_split=0.5, max_nodes=6000)
    rng = np.random.Generator(np.random.PCG64(100 + seed))
    eyes, dirs = random_rays(rng, 80, R=1.0)
    n = _leaf_seq_mismatches(cv, ray_views(eyes, dirs))
    assert n >= 70


def test_sequences_match_brute_force_shifted_canvas():
    # origin and root edge away from the unit cube: positions are in root units
    cv = trees.random_tree(2, 4, seed=7, max_nodes=3000)
    cv.origin = (-3.0, 1.0, 2.5)
    cv.root_edge = 2.0
    rng = np.random.Generator(np.random.PCG64(77))
    eyes, dirs = random_rays(rng, 60, R=4.0)
    eyes = [np.asarray(e) + np.asarray(cv.origin) for e in eyes]
    n = _leaf_seq_mismatches(cv, ray_views(eyes, dirs))
    assert n >= 50


def _node_of(cv, depth, c):
    i = c[0] // 2 ** depth + cv.R * (c[1] // 2 ** depth + cv.R * (c[2] // 2 ** depth))
    for lvl in range(depth):
        sh = depth - 1 - lvl
        o = ((c[0] >> sh) & 1) | (((c[1] >> sh) & 1) << 1) | (((c[2] >> sh) & 1) << 2)
        i = int(cv.nodes[i, 0]) + o
    return i


def _dda_exact(e, d, depth):
    """Amanatides-Woo walk of a uniform 2^depth lattice in exact rationals."""
    n = 2 ** depth
    tin, tout = F(0), None
    for k in range(3):
        ta, tb = (0 - e[k]) / d[k], (1 - e[k]) / d[k]
        lo, hi = min(ta, tb), max(ta, tb)
        tin = max(tin, lo)
        tout = hi if tout is None else min(tout, hi)
    if tin >= tout:
        return []
    p = [e[k] + tin * d[k] for k in range(3)]
    cell = []
    for k in range(3):
        c = math.floor(p[k] * n)
        if p[k] * n == c and d[k] < 0:
            c -= 1
        cell.append(min(max(c, 0), n - 1))
    t, seq = tin, []
    norm = math.sqrt(sum(float(x) ** 2 for x in d))
    while True:
        tk = [(F(cell[k] + (1 if d[k] > 0 else 0), n) - e[k]) / d[k] for k in range(3)]
        tn = min(tk)
        if sum(1 for x in tk if x == tn) > 1:
            return None  # an exact edge or corner crossing: not a unique sequence
        k = tk.index(tn)
        seq.append((tuple(cell), float(tn - t) * norm * n))
        t = tn
        cell[k] += 1 if d[k] > 0 else -1
        if not 0 <= cell[k] < n:
            return seq


@pytest.mark.parametrize("depth", [2, 3, 4])
def test_uniform_lattice_matches_exact_dda(depth):
    cv = trees.uniform_tree(1, depth, seed=depth, leaf_format=LEAF_F64)
    rng = np.random.Generator(np.random.PCG64(200 + depth))
    checked = 0
    for _ in range(40):
        e = [F(int(rng.integers(-40, 61)), 21) for _ in range(3)]
        d = [F(int(rng.choice([-1, 1]) * rng.integers(1, 30)), 7) for _ in range(3)]
        seq = _dda_exact(e, d, depth)
        if seq is None:
            continue
        dn = np.array([float(x) for x in d])
        v = ray_views([np.array([float(x) for x in e])], [dn / np.linalg.norm(dn)])
        out = oracle.render([cv], v, max_leaves=200)
        if out["flags"][0] & oracle.FLAG_NEAR_FACE:
            continue
        n = int(out["n_leaves"][0])
        assert n == len(seq)
        ids = [_node_of(cv, depth, c) for c, _ in seq]
        np.testing.assert_array_equal(out["leaf_ids"][0, :n], ids)
        np.testing.assert_allclose(out["leaf_len"][0, :n], [ln for _, ln in seq], atol=1e-12)
        np.testing.assert_array_equal(out["leaf_depth"][0, :n], depth)
        checked += 1
    assert checked >= 10


def test_chord_invariant_random_tree():
    cv = trees.random_tree(1, 7, seed=11, p_split=0.55, max_nodes=20000)
    rng = np.random.Generator(np.random.PCG64(12))
    eyes, dirs = random_rays(rng, 300)
    out = oracle.render([cv], ray_views(eyes, dirs))
    hit = out["chord"] > 0
    assert hit.sum() > 200
    tol = np.maximum(out["n_leaves"][hit], 1) * 1e-15
    assert np.all(np.abs(out["sum_len"][hit] - out["chord"][hit]) <= tol)


def test_early_termination_after_threshold_segment():
    kap = 0.3
    cv = trees.from_refinement(1, 3, lambda d, c: True,
                               lambda d, c: (0.5, 0.5, 0.5, kap), LEAF_F64)
    e, d = (-1.0, 0.3125 + 1 / 48, 0.5625 + 1 / 48), (1.0, 0.0, 0.0)
    full = oracle.render([cv], ray_views([e], [d], alpha_stop=1.0))
    stop = oracle.render([cv], ray_views([e], [d], alpha_stop=0.6))
    assert full["n_leaves"][0] == 8
    # 1 - exp(-0.3 n) >= 0.6 first holds at n = 4
    assert stop["n_leaves"][0] == 4
    assert abs(stop["rgba"][0, 3] - (1 - math.exp(-4 * kap))) < 1e-15
    amb = oracle.render([cv], ray_views([e], [d], alpha_stop=1 - math.exp(-4 * kap) + 5e-6))
    assert amb["flags"][0] & oracle.FLAG_TERM_AMBIG


def test_near_face_flags():
    cv = trees.uniform_tree(1, 2, seed=1)
    vs = ray_views([(-1.0, 0.3, 0.4), (0.25 - 0.3, 0.5 - 0.3, 0.31), (-1.0, 0.5, 0.4),
                    (-1.0, 0.31, 0.43)],
                   [(1.0, 0.0, 0.0), np.array([1.0, 1.0, 0.0]) / math.sqrt(2), (1.0, 0.0, 0.0),
                    np.array([1.0, 0.1, 0.05]) / np.linalg.norm([1.0, 0.1, 0.05])])
    out = oracle.render([cv], vs)
    assert out["flags"][0] == 0                 # generic axis ray
    assert out["flags"][1] & oracle.FLAG_NEAR_FACE  # crosses the edge x = 0.25, y = 0.5
    assert out["flags"][2] & oracle.FLAG_NEAR_FACE  # runs inside the face plane y = 0.5
    assert out["flags"][3] == 0


def test_near_face_flags_at_entry_only_and_exit_only():
    """A single cell isolates the two checks of the face band: a ray that
    enters 5e-13 from an edge of the cell and leaves far from every other
    face is flagged by its entry point alone, and one that enters far from
    the edges and leaves 5e-13 from one by its exit point alone; the same rays
    1e-9 away from the edge are not flagged."""
    cv = trees.single_cell((0.5, 0.5, 0.5), 1.0)
    d = np.array([0.3, 0.0, 1.0]) / math.hypot(0.3, 1.0)
    t_in = 1.0 / d[2]                                   # from z = -1 to the face z = 0

    def ray(x_at_entry):
        return (x_at_entry - t_in * d[0], 0.5, -1.0)

    eyes = [ray(5e-13), ray(1e-9), ray(0.7 - 5e-13), ray(0.7 - 1e-9)]
    out = oracle.render([cv], ray_views(eyes, [d] * 4))
    assert out["flags"][0] & oracle.FLAG_NEAR_FACE      # entry 5e-13 from the face x = 0
    assert out["flags"][1] == 0
    assert out["flags"][2] & oracle.FLAG_NEAR_FACE      # exit 5e-13 from the face x = 1
    assert out["flags"][3] == 0
    assert np.all(out["n_leaves"] == 1)


def test_algorithmic_bytes_hand_count():
    # uniform depth-2 lattice, axis ray through four cells: descend 2 levels to
    # the first leaf, then sibling, outer (parent boundary), sibling steps
    cv = trees.uniform_tree(1, 2, seed=1)
    out = oracle.render([cv], ray_views([(-1.0, 0.375, 0.625)], [(1.0, 0.0, 0.0)]))
    assert out["n_leaves"][0] == 4
    assert out["alg_bytes"][0] == 16 + 8 * 4 + 4 * (2 + 1)
    # coarse leaf next to a refined cell: ray enters a depth-1 leaf, then a
    # refined depth-1 cell whose depth-2 children it crosses
    cv2 = trees.from_refinement(1, 2, lambda d, c: d == 0 or (d == 1 and c == (1, 0, 1)),
                                lambda d, c: (0.1, 0.2, 0.3, 0.5), LEAF_F64)
    out = oracle.render([cv2], ray_views([(-1.0, 0.375, 0.625)], [(1.0, 0.0, 0.0)]))
    # leaves: (0,0,1)@1, then (2,1,2)@2, (3,1,2)@2: descent 1, sibling step into a
    # refined cell (+1 level), sibling step
    assert out["n_leaves"][0] == 3
    assert out["alg_bytes"][0] == 16 + 8 * 3 + 4 * (1 + (0 + 1) + 0)
    # a step that lands two levels deeper: (1,0,1)@1 and its child (2,1,2)@2
    # are refined, so after (0,0,1)@1 the ray enters (4,3,5)@3 (sibling step,
    # +2 levels), then (5,3,5)@3 (sibling), then (3,1,2)@2 (an outer face of
    # the depth-2 parent, one level up)
    cv3 = trees.from_refinement(
        1, 3, lambda d, c: d == 0 or (d == 1 and c == (1, 0, 1)) or (d == 2 and c == (2, 1, 2)),
        lambda d, c: (0.1, 0.2, 0.3, 0.5), LEAF_F64)
    out = oracle.render([cv3], ray_views([(-1.0, 0.375, 0.625)], [(1.0, 0.0, 0.0)]))
    assert out["n_leaves"][0] == 4
    assert out["alg_bytes"][0] == 16 + 8 * 4 + 4 * ((1 + 2) + 1)


def test_miss_and_eye_inside():
    cv = trees.uniform_tree(1, 2, seed=2)
    out = oracle.render([cv], ray_views([(-1.0, 0.3, 0.4), (0.3, 0.4, 0.45)],
                                        [(-1.0, 0.0, 0.0), (0.0, 0.0, 1.0)]))
    assert out["n_leaves"][0] == 0 and np.all(out["rgba"][0] == 0) and out["chord"][0] == 0
    assert out["n_leaves"][1] == 3            # z from 0.45: cells 1, 2, 3 of the column
    assert abs(out["chord"][1] - 0.55) < 1e-15
    assert abs(out["sum_len"][1] - 0.55) < 1e-15

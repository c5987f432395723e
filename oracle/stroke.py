"""Oracle of stroke application: what painting one brush stroke makes of a
canvas's leaves (Sec. 5.1 colour mix, Sec. 5.2 adaptive brush size).

TEST INFRASTRUCTURE ONLY: imported by the test-suite and the benchmark, never
by the library.  Plain Python in FP64, one leaf at a time; it shares no code
with the GPU path (nor with the canvas builder, against which it is pinned).

Optionally (`merge_uniform`) the cells the stroke left uniform are coarsened
back, without loss: a refined cell the stamps overlap whose 8 children are
leaves with identical payloads becomes one leaf of twice the optical depth
per edge, until no such cell remains.

A canvas is taken in canonical form: a dict mapping every leaf's cell
(depth, x, y, z) -- integer coordinates at that depth, the R^3 root array at
depth 0 -- to its payload tuple ((r, g, b, kappa) doubles for the F64 leaf
format; (r, g, b, a, kappa_f16_bits, pad) for RGBA8_F16).  The canvas covers
origin + [0, R root_edge)^3 in world units; a cell of depth d has edge
e = root_edge 2^-d and lower corner origin + i e.

One stroke = spherical stamps (x, y, z, r) in world units, a brush colour
rgb, an opacity density sigma per brush radius, the brush radius and a
refinement factor k.  For every leaf of the canvas, independently:

1. (Sec. 5.2) If the stamps overlap the leaf's closed box (some stamp centre
   lies at a distance < r from it), the leaf's edge exceeds radius / k and the
   leaf is above the canvas max depth, it is split into 8 children that
   inherit its colour and half its optical depth per edge; each child is
   treated again by these rules.
2. (Sec. 5.1) Otherwise, if the leaf's centre lies in a stamp (distance <= r),
   the leaf takes the stroke once: kb = sigma e / radius (the stroke's optical
   depth across the leaf), m = kb / (kb + kappa) (0 when both are 0),
   colour = m rgb + (1 - m) colour, kappa = kb + kappa.
3. RGBA8_F16 leaves are decoded (byte / 255, kappa from its half bits) before
   and encoded after: each colour byte is 255 c rounded to nearest even after
   clamping to [0, 1], A = 255 (1 - exp(-kappa)) rounded likewise, kappa to
   half through float; a child's kappa is its parent's kappa halved (in half).

The floating-point operations are written in the order stated, so that the
F64 result is exactly that of a sequential application of the same stroke.
"""
from __future__ import annotations

import math

import numpy as np

LEAF = 0x80000000
F64, RGBA8_F16 = 1, 0


def canonical_from_pool(nodes, leaves, R):
    """Leaves of a host pool (nodes (n, 2) of [child, parent], leaves array)
    as {(depth, x, y, z): payload tuple}."""
    out = {}
    stack = [(i, 0, i % R, (i // R) % R, i // (R * R)) for i in range(R ** 3)]
    while stack:
        n, d, x, y, z = stack.pop()
        c = int(nodes[n][0])
        if c & LEAF:
            out[(d, x, y, z)] = tuple(leaves[c & ~LEAF].tolist())
        else:
            for o in range(8):
                stack.append((c + o, d + 1, 2 * x + (o & 1), 2 * y + ((o >> 1) & 1),
                              2 * z + ((o >> 2) & 1)))
    return out


def _box_dist2(lo, e, s):
    d2 = 0.0
    for k in range(3):
        v = max(max(lo[k] - s[k], 0.0), s[k] - (lo[k] + e))
        d2 += v * v
    return d2


def _centre_dist2(lo, e, s):
    c = [lo[k] + 0.5 * e - s[k] for k in range(3)]
    return c[0] * c[0] + c[1] * c[1] + c[2] * c[2]


def _stroke_box(stamps):
    """Closed box around every stamp sphere (a plain speed-up: a leaf strictly
    outside it is at distance >= r from every stamp)."""
    lo = [min(s[k] - s[3] for s in stamps) for k in range(3)]
    hi = [max(s[k] + s[3] for s in stamps) for k in range(3)]
    return lo, hi


def _outside(lo, e, box):
    return any(lo[k] + e < box[0][k] or lo[k] > box[1][k] for k in range(3))


def _f16_bits(x):
    return int(np.array(np.float32(x), np.float16).view(np.uint16))


def _f16_value(bits):
    return float(np.array(bits, np.uint16).view(np.float16))


def _byte(v):
    return int(np.rint(255.0 * min(max(v, 0.0), 1.0)))


def decode(pay, fmt):
    """(r, g, b, kappa) in FP64."""
    if fmt == F64:
        return tuple(float(v) for v in pay)
    return (pay[0] / 255.0, pay[1] / 255.0, pay[2] / 255.0, _f16_value(pay[4]))


def encode(col, fmt):
    if fmt == F64:
        return tuple(col)
    kap = max(col[3], 0.0)
    a = int(np.rint(255.0 * (1.0 - math.exp(-kap))))
    return (_byte(col[0]), _byte(col[1]), _byte(col[2]), a, _f16_bits(min(kap, 65504.0)), 0)


def child_payload(pay, fmt):
    """A split leaf's child: same colour, half the optical depth per edge."""
    if fmt == F64:
        return (pay[0], pay[1], pay[2], pay[3] * 0.5)
    kap = _f16_bits(np.float32(_f16_value(pay[4])) * np.float32(0.5))
    a = int(np.rint(255.0 * (1.0 - math.exp(-_f16_value(kap)))))
    return (pay[0], pay[1], pay[2], a, kap, 0)


def paint(pay, fmt, e, rgb, sigma, radius):
    q = list(decode(pay, fmt))
    kb = sigma * e / radius
    kc = q[3]
    m = kb / (kb + kc) if kb + kc > 0.0 else 0.0
    for ch in range(3):
        q[ch] = m * rgb[ch] + (1.0 - m) * q[ch]
    q[3] = kb + kc
    return encode(q, fmt)


def apply_stroke(leaves, fmt, R, max_depth, root_edge, origin, stamps, rgb, sigma, radius, k):
    """leaves: canonical dict; stamps: (n, 4) world units.  Returns
    (new canonical dict, set of cells that were split)."""
    stamps = [tuple(float(v) for v in s) for s in np.asarray(stamps, np.float64)]
    hmin = radius / k
    out = {}
    split = set()
    box = _stroke_box(stamps)

    def visit(cell, pay):
        d, x, y, z = cell
        e = math.ldexp(root_edge, -d)
        lo = (origin[0] + x * e, origin[1] + y * e, origin[2] + z * e)
        if _outside(lo, e, box) or not any(_box_dist2(lo, e, s) < s[3] * s[3] for s in stamps):
            out[cell] = pay
            return
        if e > hmin and d < max_depth:
            split.add(cell)
            cp = child_payload(pay, fmt)
            for o in range(8):
                visit((d + 1, 2 * x + (o & 1), 2 * y + ((o >> 1) & 1), 2 * z + ((o >> 2) & 1)), cp)
            return
        if any(_centre_dist2(lo, e, s) <= s[3] * s[3] for s in stamps):
            out[cell] = paint(pay, fmt, e, rgb, sigma, radius)
        else:
            out[cell] = pay

    for cell, pay in leaves.items():
        visit(cell, pay)
    return out, split


def parent_payload(child, fmt):
    """The leaf that replaces 8 identical children: same colour, twice the
    optical depth per edge (None when that overflows the half format)."""
    if fmt == F64:
        return (child[0], child[1], child[2], child[3] * 2.0)
    kap = _f16_value(child[4]) * 2.0
    if kap > 65504.0:
        return None
    a = int(np.rint(255.0 * (1.0 - math.exp(-kap))))
    return (child[0], child[1], child[2], a, _f16_bits(kap), 0)


def merge_uniform(leaves, fmt, root_edge, origin, stamps):
    """Sec. 5.2-5.3 coarsening, read as lossless: every refined cell that the
    stamps overlap and whose 8 children are leaves with identical payloads
    becomes one leaf (same colour, twice the optical depth per edge), repeated
    until no such cell is left.  Returns (new canonical dict, merged cells)."""
    stamps = [tuple(float(v) for v in s) for s in np.asarray(stamps, np.float64)]
    box = _stroke_box(stamps)
    out = dict(leaves)
    merged = set()
    while True:
        groups = {}
        for (d, x, y, z) in out:
            if d > 0:
                groups.setdefault((d - 1, x >> 1, y >> 1, z >> 1), []).append((d, x, y, z))
        done = []
        for parent, kids in groups.items():
            if len(kids) != 8:
                continue
            pays = {out[c] for c in kids}
            if len(pays) != 1:
                continue
            d, x, y, z = parent
            e = math.ldexp(root_edge, -d)
            lo = (origin[0] + x * e, origin[1] + y * e, origin[2] + z * e)
            if _outside(lo, e, box) or not any(_box_dist2(lo, e, s) < s[3] * s[3] for s in stamps):
                continue
            pp = parent_payload(next(iter(pays)), fmt)
            if pp is not None:
                done.append((parent, kids, pp))
        if not done:
            return out, merged
        for parent, kids, pp in done:
            for c in kids:
                del out[c]
            out[parent] = pp
            merged.add(parent)


def immediate(leaves, fmt, R, max_depth, root_edge, origin, stamps, rgb, sigma, radius, k):
    """The first, immediate pass of the deferred adjustment (Sec. 5.3): every
    existing leaf whose centre lies in a stamp takes the stroke, no leaf is
    split yet.  Returns (painted dict, cells waiting for a split)."""
    stamps = [tuple(float(v) for v in s) for s in np.asarray(stamps, np.float64)]
    hmin = radius / k
    out, pending = {}, set()
    box = _stroke_box(stamps)
    for cell, pay in leaves.items():
        d, x, y, z = cell
        e = math.ldexp(root_edge, -d)
        lo = (origin[0] + x * e, origin[1] + y * e, origin[2] + z * e)
        out[cell] = pay
        if _outside(lo, e, box) or not any(_box_dist2(lo, e, s) < s[3] * s[3] for s in stamps):
            continue
        if e > hmin and d < max_depth:
            pending.add(cell)
        if any(_centre_dist2(lo, e, s) <= s[3] * s[3] for s in stamps):
            out[cell] = paint(pay, fmt, e, rgb, sigma, radius)
    return out, pending

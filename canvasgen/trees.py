"""Small hand-shaped and randomly refined canvases (input generation only).

These trees exercise the pool format directly: uniform trees of a given
depth, random refinements with abrupt depth jumps between neighbours, and
single homogeneous cells.  Payloads are drawn from a seeded PCG64 stream.
Child numbering inside a sibling group is x | y<<1 | z<<2 (Sec. 4.1.1: the
siblings of C are C+1, ... and the children of a cell that touch a face are
found by adding 2 to the first child).
"""
from __future__ import annotations

import numpy as np

from .pool import LEAF, LEAF_DTYPE, LEAF_F64, NONE, Canvas


def _quantise(rgb, kappa, leaf_format):
    n = len(kappa)
    out = np.zeros(n, LEAF_DTYPE[leaf_format])
    if leaf_format == LEAF_F64:
        out["r"], out["g"], out["b"] = rgb[:, 0], rgb[:, 1], rgb[:, 2]
        out["kappa"] = kappa
    else:
        q = np.rint(np.clip(rgb, 0.0, 1.0) * 255.0).astype(np.uint8)
        out["r"], out["g"], out["b"] = q[:, 0], q[:, 1], q[:, 2]
        out["a"] = np.rint(255.0 * (1.0 - np.exp(-kappa))).astype(np.uint8)
        k32 = np.minimum(kappa, 65504.0).astype(np.float32)
        out["kappa"] = k32.astype(np.float16).view(np.uint16)
    return out


def from_refinement(R, max_depth, refine, payload, leaf_format=LEAF_F64, root_edge=None):
    """Build a pool top-down.

    refine(depth, (ix,iy,iz)) -> bool decides whether a cell is split;
    payload(depth, (ix,iy,iz)) -> (r, g, b, kappa) gives a leaf's values.
    Groups are emitted breadth first.
    """
    R3 = R ** 3
    P0 = (R3 + 7) // 8 * 8
    child = [LEAF] * P0
    parent = [NONE] * P0
    cells = [None] * P0
    for z in range(R):
        for y in range(R):
            for x in range(R):
                cells[x + R * (y + R * z)] = (0, (x, y, z))
    rgb, kap = [], []
    queue = list(range(R3))
    head = 0
    leaf_of = {}
    while head < len(queue):
        i = queue[head]
        head += 1
        d, (x, y, z) = cells[i]
        if d < max_depth and refine(d, (x, y, z)):
            g = len(child)
            child[i] = g
            for o in range(8):
                child.append(LEAF)
                parent.append(i)
                cells.append((d + 1, (2 * x + (o & 1), 2 * y + ((o >> 1) & 1), 2 * z + ((o >> 2) & 1))))
                queue.append(g + o)
        else:
            leaf_of[i] = len(rgb)
            v = payload(d, (x, y, z))
            rgb.append(v[:3])
            kap.append(v[3])
    for i, li in leaf_of.items():
        child[i] = LEAF | li
    for i in range(R3, P0):
        child[i] = LEAF | 0
    nodes = np.stack([np.asarray(child, np.uint64), np.asarray(parent, np.uint64)], 1).astype(np.uint32)
    leaves = _quantise(np.asarray(rgb, np.float64).reshape(-1, 3), np.asarray(kap, np.float64),
                       leaf_format)
    return Canvas(nodes, leaves, R, max_depth, leaf_format, root_edge=root_edge)


def uniform_tree(R, depth, seed=0, leaf_format=LEAF_F64, kappa_range=(0.0, 2.0)):
    """Every cell refined to exactly `depth`; random per-leaf payload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return from_refinement(
        R, depth, lambda d, c: d < depth,
        lambda d, c: (*rng.uniform(0, 1, 3), rng.uniform(*kappa_range)), leaf_format)


def random_tree(R, max_depth, seed=0, p_split=0.45, leaf_format=LEAF_F64, kappa_range=(0.0, 2.0),
                max_nodes=20000):
    """Random refinement: a cell splits with probability p_split (always at depth 0 for R=1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    budget = [max_nodes]

    def refine(d, c):
        if budget[0] <= 8:
            return False
        s = d == 0 or rng.uniform() < p_split
        if s:
            budget[0] -= 8
        return s

    return from_refinement(R, max_depth, refine,
                           lambda d, c: (*rng.uniform(0, 1, 3), rng.uniform(*kappa_range)),
                           leaf_format)


def deep_path_tree(max_depth, target=(0.3, 0.6, 0.45), seed=0, leaf_format=LEAF_F64,
                   kappa_range=(0.0, 1.0), halo=0):
    """One root refined along a single path down to max_depth around `target`.

    With halo > 0 the cells within `halo` cells of the path cell (same depth)
    are refined too, giving long same-depth runs next to abrupt depth jumps.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.asarray(target, np.float64)

    def refine(d, c):
        h = 2.0 ** -d
        tc = np.floor(t / h).astype(np.int64)
        return all(abs(int(c[a]) - int(tc[a])) <= halo for a in range(3))

    return from_refinement(1, max_depth, refine,
                           lambda d, c: (*rng.uniform(0, 1, 3), rng.uniform(*kappa_range)),
                           leaf_format)


def single_cell(rgb, kappa, leaf_format=LEAF_F64):
    """A canvas that is one homogeneous root leaf."""
    return from_refinement(1, 0, lambda d, c: False, lambda d, c: (*rgb, kappa), leaf_format)

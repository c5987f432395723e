"""Brute-force leaf sequences for tiny canvases (pins the oracle's traversal).

Every leaf box is computed from the pool by a breadth-first walk (children
x | y<<1 | z<<2), every box is slab-tested against the ray, positive-length
intersections inside the canvas chord are kept and sorted by entry t.  No
descent, no neighbour stepping, no restart: it shares nothing with the
oracle's traversal.
"""
from __future__ import annotations

import numpy as np

LEAF = 0x80000000


def leaf_boxes(canvas):
    """Return (node_ids, lo (n,3), h (n,), depth (n,)) in root-edge units."""
    R = canvas.R
    nodes = canvas.nodes
    ids, los, hs, deps = [], [], [], []
    frontier = []
    for z in range(R):
        for y in range(R):
            for x in range(R):
                frontier.append((x + R * (y + R * z), 0, np.array([x, y, z], np.float64)))
    while frontier:
        nxt = []
        for i, d, lo in frontier:
            c = int(nodes[i, 0])
            h = 2.0 ** -d
            if c & LEAF:
                ids.append(i)
                los.append(lo)
                hs.append(h)
                deps.append(d)
            else:
                for o in range(8):
                    off = np.array([o & 1, (o >> 1) & 1, (o >> 2) & 1], np.float64) * (h / 2)
                    nxt.append((c + o, d + 1, lo + off))
        frontier = nxt
    return np.array(ids, np.int64), np.array(los), np.array(hs), np.array(deps)


def sequence(canvas, boxes, eye_world, d, min_len=1e-13):
    """Leaves hit by the ray with positive length, ordered by entry t.

    Returns (node_ids, local lengths l = segment / leaf edge)."""
    ids, lo, h, _ = boxes
    o = (np.asarray(eye_world, np.float64) - np.asarray(canvas.origin)) / canvas.root_edge
    d = np.asarray(d, np.float64)
    R = float(canvas.R)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        # canvas chord
        ta, tb = (0.0 - o) * inv, (R - o) * inv
        t_in_c = np.max(np.where(d != 0, np.minimum(ta, tb), -np.inf))
        t_out_c = np.min(np.where(d != 0, np.maximum(ta, tb), np.inf))
        if np.any((d == 0) & ((o < 0) | (o > R))):
            return np.zeros(0, np.int64), np.zeros(0)
        t0, t1 = max(t_in_c, 0.0), t_out_c
        if not t0 < t1:
            return np.zeros(0, np.int64), np.zeros(0)
        a = (lo - o[None, :]) * inv[None, :]
        b = (lo + h[:, None] - o[None, :]) * inv[None, :]
        par_inside = (lo <= o[None, :]) & (o[None, :] <= lo + h[:, None])
        tmin = np.where(d[None, :] != 0, np.minimum(a, b), np.where(par_inside, -np.inf, np.inf))
        tmax = np.where(d[None, :] != 0, np.maximum(a, b), np.where(par_inside, np.inf, -np.inf))
    t_in = np.maximum(np.max(tmin, axis=1), t0)
    t_out = np.minimum(np.min(tmax, axis=1), t1)
    keep = t_out - t_in > min_len
    order = np.argsort(t_in[keep], kind="stable")
    sel = np.nonzero(keep)[0][order]
    return ids[sel], (t_out[sel] - t_in[sel]) / h[sel]

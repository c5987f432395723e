"""Host model of pool edits (test infrastructure).

Applies PAINT / REFINE / COARSEN edits to a host pool (nodes (n, 2) of
[child, parent], leaves) with the allocation rule of the C-ABI: a refined
leaf's children take the most recently freed group, else 8 new ids at the
end of the pool (rounded up to a multiple of 8).  The result is an ordinary
pool that the oracle traces and cvx_upload_pool accepts, so an edited device
pool can be compared with the oracle and with a fresh upload.
"""
from __future__ import annotations

import numpy as np

from canvasgen.pool import LEAF, LEAF_DTYPE, LEAF_F64, LEAF_RGBA8_F16, NONE, Canvas

PAINT, REFINE, COARSEN = 0, 1, 2


def payload_f64(rng):
    return np.array((rng.uniform(), rng.uniform(), rng.uniform(), rng.uniform(0, 3)),
                    LEAF_DTYPE[LEAF_F64])[()]


def payload_rgba8(rng):
    r, g, b = (int(x) for x in rng.integers(0, 256, 3))
    k = int(np.float16(rng.uniform(0, 3)).view(np.uint16))
    return np.array((r, g, b, 255, k, 0), LEAF_DTYPE[LEAF_RGBA8_F16])[()]


class PoolModel:
    def __init__(self, cv: Canvas):
        self.R, self.max_depth, self.fmt = cv.R, cv.max_depth, cv.leaf_format
        self.origin, self.root_edge = cv.origin, cv.root_edge
        self.child = [int(x) for x in cv.nodes[:, 0]]
        self.parent = [int(x) for x in cv.nodes[:, 1]]
        self.leaves = [cv.leaves[i] for i in range(len(cv.leaves))]
        self.free = []                      # freed groups, LIFO
        self.state = {}                     # node -> depth for nodes in the tree
        R3 = self.R ** 3
        stack = [(i, 0) for i in range(R3)]
        while stack:
            i, d = stack.pop()
            self.state[i] = d
            if not (self.child[i] & LEAF):
                stack.extend((self.child[i] + o, d + 1) for o in range(8))

    # -- queries --------------------------------------------------------------
    def is_leaf(self, i):
        return i in self.state and bool(self.child[i] & LEAF)

    def is_refined(self, i):
        return i in self.state and not (self.child[i] & LEAF)

    def leaves_list(self):
        return [i for i in self.state if self.child[i] & LEAF]

    def coarsenable(self):
        return [i for i in self.state if not (self.child[i] & LEAF)
                and all(self.child[self.child[i] + o] & LEAF for o in range(8))]

    # -- edits ----------------------------------------------------------------
    def _new_leaf(self, payload):
        self.leaves.append(payload)
        return LEAF | (len(self.leaves) - 1)

    def apply(self, edits, payloads):
        """Returns the first child id per edit (NONE when not REFINE)."""
        out = []
        for op, node, fp in edits:
            if op == PAINT:
                assert self.is_leaf(node)
                self.child[node] = self._new_leaf(payloads[fp])
                out.append(NONE)
            elif op == REFINE:
                assert self.is_leaf(node) and self.state[node] + 1 <= self.max_depth
                if self.free:
                    g = self.free.pop()
                else:
                    g = (len(self.child) + 7) // 8 * 8
                    while len(self.child) < g + 8:
                        self.child.append(LEAF)
                        self.parent.append(NONE)
                self.child[node] = g
                for o in range(8):
                    self.child[g + o] = self._new_leaf(payloads[fp + o])
                    self.parent[g + o] = node
                    self.state[g + o] = self.state[node] + 1
                out.append(g)
            elif op == COARSEN:
                g = self.child[node]
                assert self.is_refined(node) and all(self.child[g + o] & LEAF for o in range(8))
                for o in range(8):
                    del self.state[g + o]
                self.child[node] = self._new_leaf(payloads[fp])
                self.free.append(g)
                out.append(NONE)
            else:
                raise ValueError(op)
        return np.array(out, np.uint32)

    def canvas(self) -> Canvas:
        nodes = np.stack([np.array(self.child, np.uint32), np.array(self.parent, np.uint32)], 1)
        leaves = np.array(self.leaves, dtype=self.leaves[0].dtype) if self.leaves else None
        return Canvas(nodes, leaves, self.R, self.max_depth, self.fmt, origin=self.origin,
                      root_edge=self.root_edge)


def random_edits(model: PoolModel, rng, n, payload_of, p=(0.5, 0.3, 0.2)):
    """n random valid edits against the model (applied to it as they are drawn);
    returns (edits, payloads, expected first children)."""
    edits, payloads, firsts = [], [], []
    for _ in range(n):
        op = int(rng.choice(3, p=p))
        if op == COARSEN:
            cand = model.coarsenable()
            if not cand:
                op = PAINT
        if op == REFINE:
            cand = [i for i in model.leaves_list() if model.state[i] < model.max_depth]
            if not cand:
                op = PAINT
        if op == PAINT:
            cand = model.leaves_list()
        node = int(cand[int(rng.integers(len(cand)))])
        k = 8 if op == REFINE else 1
        fp = len(payloads)
        payloads.extend(payload_of(rng) for _ in range(k))
        firsts.extend(model.apply([(op, node, 0)], payloads[fp:fp + k]))
        edits.append((op, node, fp))
    return edits, payloads, np.array(firsts, np.uint32)

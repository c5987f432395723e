"""The outer-face neighbour links (G_3, Sec. 4.1.1-4.1.2) the GPU derives,
against point location.

For a cell of depth d >= 1 with integer coordinates c (depth-d cells of the
R 2^d lattice), the outer face on axis k is the face it shares with its
parent: the high face when its octant bit on k is 1, the low face when it is
0.  Its link is the cell containing the point just across the centre of that
face: located from the roots by the coordinates' bits, that is the depth-d
cell at c +- e_k when it exists (leaf or refined), else the coarser leaf that
covers it, and none (0xffffffff) past the canvas boundary.  Roots carry no
links.  The tree structure is read from the device records themselves
(x = first child, or 1 | depth << 1 for a leaf), so the check also covers
pools after edits and strokes, whose links the library rebuilds locally.
"""
import numpy as np
import pytest

from canvasgen import LEAF_F64, LEAF_RGBA8_F16, trees
from canvasgen.pool import LEAF_DTYPE
from canvasgen.strokes import gen_strokes

from editmodel import PoolModel, payload_rgba8, random_edits

NONE = 0xFFFFFFFF


def _walk(x_words, R):
    """{node: (depth, cx, cy, cz)} of every node reachable from the roots."""
    out = {}
    stack = [(i, 0, (i % R, (i // R) % R, i // (R * R))) for i in range(R ** 3)]
    while stack:
        n, d, c = stack.pop()
        out[n] = (d, c)
        x = int(x_words[n])
        if not x & 1:
            for o in range(8):
                stack.append((x + o, d + 1, tuple(2 * c[k] + ((o >> k) & 1) for k in range(3))))
    return out


def _locate(x_words, R, d, c):
    """Node covering the depth-d cell c: the depth-d node, or the coarser leaf."""
    r = [c[k] >> d for k in range(3)]
    n = r[0] + R * (r[1] + R * r[2])
    for lv in range(1, d + 1):
        x = int(x_words[n])
        if x & 1:
            return n
        n = x + sum(((c[k] >> (d - lv)) & 1) << k for k in range(3))
    return n


def expected_links(x_words, R):
    """{node: (link_x, link_y, link_z)} by point location across each outer face."""
    out = {}
    for n, (d, c) in _walk(x_words, R).items():
        if d == 0:
            out[n] = (NONE, NONE, NONE)
            continue
        links = []
        for k in range(3):
            nb = list(c)
            nb[k] += 1 if c[k] & 1 else -1
            links.append(NONE if not 0 <= nb[k] < (R << d) else _locate(x_words, R, d, nb))
        out[n] = tuple(links)
    return out


def check_records(rec, R):
    """Every reachable node's leaf depth and three links; returns the count."""
    walk = _walk(rec[:, 0], R)
    want = expected_links(rec[:, 0], R)
    bad = []
    for n, (d, _) in walk.items():
        x = int(rec[n, 0])
        if x & 1 and x != (1 | (d << 1)):
            bad.append((n, "depth", x, d))
        got = tuple(int(v) for v in rec[n, 1:4])
        if got != want[n]:
            bad.append((n, walk[n], got, want[n]))
    assert not bad, (len(bad), bad[:4])
    return len(walk)


# ---- the rule itself, on hand-derived cases (CPU) -------------------------

def test_rule_on_hand_derived_cases():
    # R = 1, root refined once, child 3 (x=1, y=1, z=0) refined again
    x = np.full(24, 1, np.int64)      # leaves by default
    x[0] = 8                          # root -> children 8..15
    x[8 + 3] = 16                     # child 3 -> grandchildren 16..23
    x[1:8] = NONE                     # padding slots, unreachable
    links = expected_links(x, 1)
    # depth 1: every outer face of a child of the single root is the canvas boundary
    for n in range(8, 16):
        assert links[n] == (NONE, NONE, NONE), n
    # grandchild 16 = octant 0 of child 3 (x=2, y=2, z=0 at depth 2): its low x
    # face borders depth-2 cell (1, 2, 0), inside the unrefined child 2 (x=0,
    # y=1): the coarser leaf 10; its low y face borders (2, 1, 0), inside
    # child 1 (x=1, y=0): leaf 9; its low z face is the canvas boundary
    assert links[16] == (10, 9, NONE)
    # grandchild 23 = octant 7 (x=3, y=3, z=1): high x and y faces are the
    # boundary; its high z face borders (3, 3, 2), inside child 7: leaf 15
    assert links[23] == (NONE, NONE, 15)
    # R = 2, two refined roots side by side on x: root 0's child with x bit 1
    # links across x to root 1's child with x bit 0 (same y, z)
    x = np.full(24, 1, np.int64)
    x[0], x[1] = 8, 16
    links = expected_links(x, 2)
    assert links[8 + 1][0] == 16 + 0
    assert links[16 + 0][0] == 8 + 1
    assert links[8 + 0][0] == NONE    # low x face of the canvas
    # root 2 (y=1, a leaf): root 0's children with y bit 1 link across y to it
    assert links[8 + 2][1] == 2 and links[8 + 7][1] == 2


# ---- GPU-built links (through the C-ABI) --------------------------------

@pytest.fixture(scope="module")
def sess():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_02724_amd.session import Session
    s = Session(0)
    yield s
    s.close()


@pytest.mark.gpu
@pytest.mark.parametrize("R,depth,seed", [(1, 6, 91), (2, 5, 92), (3, 4, 93), (4, 4, 94),
                                          (1, 12, 95)])
def test_upload_links_match_point_location(sess, R, depth, seed):
    from paper_1704_02724_amd import cvx
    cv = trees.random_tree(R, depth, seed=seed, max_nodes=20000, leaf_format=LEAF_RGBA8_F16)
    sess.upload(0, cv)
    rec = cvx.cvx_read_records(sess.ctx, 0)
    assert check_records(rec, R) > R ** 3


@pytest.mark.gpu
def test_links_after_edits_and_a_stroke_match_point_location(sess):
    from paper_1704_02724_amd import cvx
    cv = trees.random_tree(2, 6, seed=96, max_nodes=8000, leaf_format=LEAF_RGBA8_F16)
    m = PoolModel(cv)
    sess.upload(0, cv)
    rng = np.random.Generator(np.random.PCG64(96))
    for p in [(0.2, 0.7, 0.1), (0.3, 0.3, 0.4), (0.3, 0.5, 0.2)]:
        edits, payloads, _ = random_edits(m, rng, 120, payload_rgba8, p=p)
        sess.edit(0, edits, np.array(payloads, dtype=LEAF_DTYPE[LEAF_RGBA8_F16]))
        check_records(cvx.cvx_read_records(sess.ctx, 0), 2)
    st = gen_strokes(rng, 1, -6, -5)
    small = trees.random_tree(1, 4, seed=97, max_nodes=600, leaf_format=LEAF_F64)
    small.max_depth = 9               # room for the stroke's splits
    sess.upload(1, small)
    pending = sess.stroke_begin(1, st.stamps_of(0), st.rgb[0], st.sigma[0], st.radius[0], 4.0)
    steps = 0
    while pending and steps < 40:
        pending = sess.stroke_step(1)
        steps += 1
    assert pending == 0 and steps > 0
    check_records(cvx.cvx_read_records(sess.ctx, 1), 1)

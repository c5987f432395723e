"""CPU pins of the pool-edit model used by the GPU edit tests: the pools it
produces are valid, refining a leaf into eight children of half the optical
depth leaves every image unchanged, and a coarsening undoes a refinement."""
import numpy as np
import pytest

from canvasgen import LEAF_F64, LEAF_RGBA8_F16, trees
from canvasgen.pool import LEAF_DTYPE
from oracle import oracle

from editmodel import (COARSEN, PAINT, REFINE, PoolModel, payload_f64, payload_rgba8,
                       random_edits)
from helpers import random_rays, ray_views


@pytest.fixture(scope="module")
def cvx():
    from paper_1704_02724_amd import cvx as mod
    return mod


def test_random_edits_give_valid_pools(cvx):
    rng = np.random.Generator(np.random.PCG64(71))
    for R, depth, fmt, pay in [(1, 6, LEAF_RGBA8_F16, payload_rgba8), (2, 5, LEAF_F64, payload_f64)]:
        cv = trees.random_tree(R, depth, seed=71 + R, max_nodes=3000, leaf_format=fmt)
        m = PoolModel(cv)
        for _ in range(4):
            random_edits(m, rng, 30, pay)
            out = m.canvas()
            d = cvx.make_desc(out.origin, out.root_edge, out.R, out.max_depth, out.leaf_format)
            rc, msg = cvx.cvx_validate_pool(d, out.nodes, out.leaves)
            assert rc == cvx.CVX_OK, msg


def test_refine_with_half_kappa_keeps_the_image():
    cv = trees.random_tree(1, 4, seed=72, max_nodes=2000, leaf_format=LEAF_F64)
    m = PoolModel(cv)
    rng = np.random.Generator(np.random.PCG64(72))
    eyes, dirs = random_rays(rng, 300)
    vs = ray_views(eyes, dirs)
    before = oracle.render([m.canvas()], vs)
    edits, pays = [], []
    for node in [i for i in m.leaves_list() if m.state[i] < m.max_depth][:20]:
        lf = m.leaves[m.child[node] & 0x7FFFFFFF]
        half = np.array((lf["r"], lf["g"], lf["b"], lf["kappa"] / 2), LEAF_DTYPE[LEAF_F64])[()]
        edits.append((REFINE, node, len(pays)))
        pays.extend([half] * 8)
    m.apply(edits, pays)
    after = oracle.render([m.canvas()], vs)
    np.testing.assert_allclose(after["rgba"], before["rgba"], atol=1e-12)
    assert after["n_leaves"].sum() > before["n_leaves"].sum()


def test_coarsen_undoes_refine_and_reuses_the_group():
    cv = trees.random_tree(1, 3, seed=73, max_nodes=500, leaf_format=LEAF_F64)
    m = PoolModel(cv)
    rng = np.random.Generator(np.random.PCG64(73))
    eyes, dirs = random_rays(rng, 200)
    vs = ray_views(eyes, dirs)
    before = oracle.render([m.canvas()], vs)
    refinable = [i for i in m.leaves_list() if m.state[i] < m.max_depth]
    node = refinable[0]
    orig = m.leaves[m.child[node] & 0x7FFFFFFF]
    n0 = len(m.child)
    g = m.apply([(REFINE, node, 0)], [payload_f64(rng) for _ in range(8)])[0]
    assert g % 8 == 0 and g >= n0 - (n0 % 8)
    m.apply([(COARSEN, node, 0)], [orig])
    after = oracle.render([m.canvas()], vs)
    np.testing.assert_array_equal(after["rgba"], before["rgba"])
    other = [i for i in refinable if i != node][0]
    g2 = m.apply([(REFINE, other, 0)], [payload_f64(rng) for _ in range(8)])[0]
    assert g2 == g                                  # the freed group is reused first
    m.apply([(PAINT, g2 + 3, 0)], [orig])
    assert m.is_leaf(g2 + 3)

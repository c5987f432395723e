"""GPU pool edits (cvx_edit_pool) against the host edit model: after every
batch of random PAINT / REFINE / COARSEN edits the device pool renders
bit-identically to a fresh upload of the model's pool, its first-child ids
are the model's, and its leaf sequences and colours match the oracle on the
model's pool.  Rejected batches change nothing."""
import numpy as np
import pytest

from canvasgen import LEAF_F64, LEAF_RGBA8_F16, make_view, trees
from canvasgen.pool import LEAF_DTYPE
from oracle import oracle

from editmodel import (COARSEN, PAINT, REFINE, PoolModel, payload_f64, payload_rgba8,
                       random_edits)
from gpu_common import all_ray_ids, compare_traces, rgba_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sess():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_02724_amd.session import Session
    s = Session(0)
    yield s
    s.close()


def _views(rng, n, W, H, canvas_id=0):
    vs, off = [], 0
    for _ in range(n):
        e = rng.uniform(0.05, 0.95, 3)
        tgt = rng.uniform(0.2, 0.8, 3)
        vs.append(make_view(e, tgt - e, rng.uniform(0.4, 1.2), W, H, canvas_id=canvas_id,
                            out_offset_px=off))
        off += W * H
    return vs


def _pays(payloads, fmt):
    return np.array(payloads, dtype=LEAF_DTYPE[fmt])


def _check_against_model(sess, m, views, variant, tol):
    from paper_1704_02724_amd import cvx
    exp = m.canvas()
    assert cvx.cvx_pool_nodes(sess.ctx, 0) == exp.n_nodes
    sess.upload(1, exp)
    # every record word and every outer-face link equals a fresh upload's
    np.testing.assert_array_equal(cvx.cvx_read_records(sess.ctx, 0),
                                  cvx.cvx_read_records(sess.ctx, 1))
    a = sess.render(views, variant).cpu().numpy()
    b = sess.render([dict(v, canvas_id=1) for v in views], variant).cpu().numpy()
    np.testing.assert_array_equal(a, b)
    ids = all_ray_ids(views)
    orc = oracle.render([exp], views, ids, max_leaves=512)
    gpu = sess.trace(views, ids, 512, variant)
    assert np.all((gpu["flags"] & 0x5) == 0)
    cmp = compare_traces(orc, gpu, 512)
    assert cmp["seq_mismatch"] == 0, cmp
    assert rgba_err(a, orc["rgba"], cmp["ok_mask"]) <= tol
    return a


@pytest.mark.parametrize("R,depth,fmt,variant,seed", [
    (1, 7, LEAF_RGBA8_F16, "fp32_rebased", 81),
    (2, 5, LEAF_RGBA8_F16, "fp32_rebased", 82),
    (1, 6, LEAF_F64, "fp64_plain", 83),
])
def test_edits_match_model_upload_and_oracle(sess, R, depth, fmt, variant, seed):
    cv = trees.random_tree(R, depth, seed=seed, max_nodes=6000, leaf_format=fmt)
    m = PoolModel(cv)
    sess.upload(0, cv)
    rng = np.random.Generator(np.random.PCG64(seed))
    views = _views(rng, 2, 40, 32)
    pay = payload_rgba8 if fmt == LEAF_RGBA8_F16 else payload_f64
    tol = 1e-3 if variant == "fp32_rebased" else 1e-6  # float32 image
    for rnd, p in enumerate([(0.3, 0.6, 0.1), (0.4, 0.2, 0.4), (0.5, 0.3, 0.2)]):
        edits, payloads, firsts = random_edits(m, rng, 80, pay, p=p)
        got = sess.edit(0, edits, _pays(payloads, fmt))
        np.testing.assert_array_equal(got, firsts)
        _check_against_model(sess, m, views, variant, tol)


def test_pool_grows_and_reuses_freed_groups(sess):
    from paper_1704_02724_amd import cvx
    cv = trees.random_tree(1, 3, seed=85, max_nodes=200, leaf_format=LEAF_RGBA8_F16)
    cv.max_depth = 9
    m = PoolModel(cv)
    sess.upload(0, cv)
    rng = np.random.Generator(np.random.PCG64(85))
    views = _views(rng, 1, 48, 40)
    n0 = cvx.cvx_pool_nodes(sess.ctx, 0)
    for _ in range(4):              # mostly refinements: the pool grows past its capacity
        edits, payloads, firsts = random_edits(m, rng, 150, payload_rgba8, p=(0.1, 0.85, 0.05))
        np.testing.assert_array_equal(sess.edit(0, edits, _pays(payloads, LEAF_RGBA8_F16)), firsts)
    assert cvx.cvx_pool_nodes(sess.ctx, 0) > 8 * n0
    _check_against_model(sess, m, views, "fp32_rebased", 1e-3)
    # coarsen a few groups, then refine: the freed groups come back LIFO
    nodes = m.coarsenable()[:3]
    edits = [(COARSEN, n, i) for i, n in enumerate(nodes)]
    pays = [payload_rgba8(rng) for _ in nodes]
    freed = [m.child[n] for n in nodes]
    m.apply(edits, pays)
    sess.edit(0, edits, _pays(pays, LEAF_RGBA8_F16))
    leaves = [i for i in m.leaves_list() if m.state[i] < m.max_depth][:3]
    edits = [(REFINE, n, 8 * i) for i, n in enumerate(leaves)]
    pays = [payload_rgba8(rng) for _ in range(8 * len(leaves))]
    firsts = m.apply(edits, pays)
    assert list(firsts) == freed[::-1]
    np.testing.assert_array_equal(sess.edit(0, edits, _pays(pays, LEAF_RGBA8_F16)), firsts)
    _check_against_model(sess, m, views, "fp32_rebased", 1e-3)


def test_edits_next_to_deep_subtrees(sess):
    """Refine, then coarsen again, every shallow leaf of a tree refined along
    one path to depth 14: the deep cells next to them link to them as their
    coarser neighbours, so their links must follow both changes."""
    from paper_1704_02724_amd import cvx
    cv = trees.deep_path_tree(14, seed=87, leaf_format=LEAF_RGBA8_F16, halo=1)
    m = PoolModel(cv)
    sess.upload(0, cv)
    rng = np.random.Generator(np.random.PCG64(87))
    views = _views(rng, 2, 32, 32)
    shallow = sorted(i for i in m.leaves_list() if m.state[i] <= 4)
    assert len(shallow) > 20
    edits = [(REFINE, n, 8 * i) for i, n in enumerate(shallow)]
    pays = [payload_rgba8(rng) for _ in range(8 * len(shallow))]
    np.testing.assert_array_equal(sess.edit(0, edits, _pays(pays, LEAF_RGBA8_F16)),
                                  m.apply(edits, pays))
    _check_against_model(sess, m, views, "fp32_rebased", 1e-3)
    edits = [(COARSEN, n, i) for i, n in enumerate(shallow)]
    pays = [payload_rgba8(rng) for _ in shallow]
    m.apply(edits, pays)
    sess.edit(0, edits, _pays(pays, LEAF_RGBA8_F16))
    _check_against_model(sess, m, views, "fp32_rebased", 1e-3)


def test_rejected_edits_change_nothing(sess):
    from paper_1704_02724_amd import cvx
    cv = trees.random_tree(1, 4, seed=86, max_nodes=3000, leaf_format=LEAF_RGBA8_F16)
    m = PoolModel(cv)
    sess.upload(0, cv)
    rng = np.random.Generator(np.random.PCG64(86))
    views = _views(rng, 1, 32, 24)
    ref = sess.render(views).cpu().numpy()
    n0 = cvx.cvx_pool_nodes(sess.ctx, 0)
    rec0 = cvx.cvx_read_records(sess.ctx, 0)
    leaves = [i for i in m.leaves_list() if m.state[i] < m.max_depth]
    deepest = [i for i in m.leaves_list() if m.state[i] == m.max_depth]
    internal = [i for i in m.state if m.is_refined(i)]
    good = [payload_rgba8(rng) for _ in range(8)]
    neg = np.array(good, dtype=LEAF_DTYPE[LEAF_RGBA8_F16])
    neg["kappa"][0] = 0xBC00                        # -1.0 in half precision
    inf = np.array(good, dtype=LEAF_DTYPE[LEAF_RGBA8_F16])
    inf["kappa"][0] = 0x7C00                        # +inf
    P = _pays(good, LEAF_RGBA8_F16)
    cases = [
        ([(PAINT, internal[0], 0)], P),                       # paint a refined node
        ([(COARSEN, leaves[0], 0)], P),                       # coarsen a leaf
        ([(PAINT, n0 + 100, 0)], P),                          # node out of range
        ([(PAINT, leaves[0], 8)], P),                         # payload index out of range
        ([(REFINE, leaves[0], 1)], P),                        # needs 8 payloads from 1
        ([(PAINT, leaves[0], 0)], neg),                       # negative kappa
        ([(PAINT, leaves[0], 0)], inf),                       # infinite kappa
        ([(7, leaves[0], 0)], P),                             # unknown op
        ([(REFINE, leaves[0], 0), (PAINT, leaves[0], 0)], P),  # leaves[0] is refined by then
        ([(PAINT, leaves[1], 0), (REFINE, leaves[2], 0), (COARSEN, leaves[1], 0)], P),
    ]
    if deepest:
        cases.append(([(REFINE, deepest[0], 0)], P))          # beyond the max depth
    for edits, pays in cases:
        with pytest.raises(cvx.CvxError) as e:
            sess.edit(0, edits, pays)
        assert e.value.code == cvx.CVX_ERR_INVALID_ARG, edits
        np.testing.assert_array_equal(sess.render(views).cpu().numpy(), ref)
        assert cvx.cvx_pool_nodes(sess.ctx, 0) == n0
        np.testing.assert_array_equal(cvx.cvx_read_records(sess.ctx, 0), rec0)
    # a freed node is no longer in the tree
    node = leaves[3]
    g = sess.edit(0, [(REFINE, node, 0)], P)[0]
    lf = m.leaves[m.child[node] & 0x7FFFFFFF]
    sess.edit(0, [(COARSEN, node, 0)], _pays([lf], LEAF_RGBA8_F16))
    np.testing.assert_array_equal(sess.render(views).cpu().numpy(), ref)
    with pytest.raises(cvx.CvxError) as e:
        sess.edit(0, [(PAINT, int(g) + 2, 0)], P)
    assert e.value.code == cvx.CVX_ERR_INVALID_ARG

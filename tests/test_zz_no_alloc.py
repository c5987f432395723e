"""The allocation-free render entry point against cvx_render, through the C-ABI.

cvx_render_noalloc stages its view table and queue header in the library's
fixed device array instead of context-allocated memory; it runs the same
kernels, so its images must equal cvx_render's bit for bit.  Two calls in a
row, the second with fewer and smaller views, check that the array's
contents from the first call do not leak into the second.
"""
import numpy as np
import pytest

from canvasgen import LEAF_RGBA8_F16, configs, make_view, trees

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


def _views(rng, specs):
    vs, off = [], 0
    for canvas_id, W, H in specs:
        e = rng.uniform(0.1, 0.9, 3)
        tgt = rng.uniform(0.3, 0.7, 3)
        vs.append(make_view(e, tgt - e, rng.uniform(0.4, 1.0), W, H, canvas_id=canvas_id,
                            out_offset_px=off))
        off += W * H
    return vs


def _both(sess, views, **kw):
    torch = sess.torch
    n = sess.out_pixels(views)
    ref = torch.full((n, 4), -1.0, dtype=torch.float32, device=sess.device)
    img = torch.full((n, 4), -2.0, dtype=torch.float32, device=sess.device)
    sref, simg = sess.new_stats(), sess.new_stats()
    sess.render(views, out=ref, stats=sref, **kw)
    sess.render(views, out=img, stats=simg, noalloc=True, **kw)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), img.cpu().numpy(), sref.cpu().numpy(), simg.cpu().numpy()


def test_noalloc_equals_render_twice_shrinking(sess):
    w = configs.tiny(leaf_format=LEAF_RGBA8_F16, W=8, H=8)
    sess.upload(0, w.canvases[0])
    sess.upload(1, trees.random_tree(2, 6, seed=71, max_nodes=60000,
                                     leaf_format=LEAF_RGBA8_F16))
    rng = np.random.Generator(np.random.PCG64(72))
    first = _views(rng, [(0, 160, 120), (1, 96, 200), (0, 77, 51), (1, 130, 66)])
    second = _views(rng, [(1, 40, 24)])
    for views in (first, second):
        ref, img, sref, simg = _both(sess, views)
        assert np.isfinite(ref).all() and (ref[:, 3] > 0).any()
        np.testing.assert_array_equal(img, ref)
        np.testing.assert_array_equal(simg, sref)
    # with a tuned launch shape, eye inside the canvas (shared first leaf) or not
    for kw in (dict(tile=(16, 4), wg_size=64, workgroups=37),
               dict(tile=(4, 16), wg_size=256, single_queue=1, per_ray_start=1),
               dict(rays_per_wave=256, refill_min=16)):
        for views in (first, second):
            ref, img, _, _ = _both(sess, views, **kw)
            np.testing.assert_array_equal(img, ref)


def test_noalloc_limits(sess):
    from paper_1704_02724_amd import cvx
    w = configs.tiny(leaf_format=LEAF_RGBA8_F16, W=8, H=8)
    sess.upload(0, w.canvases[0])
    too_many = [make_view((0.5, 0.5, -1.0), (0.0, 0.0, 1.0), 0.5, 4, 4, out_offset_px=16 * i)
                for i in range(cvx.CVX_NOALLOC_MAX_VIEWS + 1)]
    out = sess.torch.zeros((16 * len(too_many), 4), dtype=sess.torch.float32,
                           device=sess.device)
    varr = cvx.make_views(too_many)
    with pytest.raises(cvx.CvxError) as e:
        cvx.cvx_render_noalloc(sess.ctx, varr, out.data_ptr(), cvx.make_opts())
    assert e.value.code == cvx.CVX_ERR_INVALID_ARG
    assert "CVX_NOALLOC_MAX_VIEWS" in str(e.value)
    for bad in (dict(use_graph=True), dict(chord_pieces=2)):
        with pytest.raises(cvx.CvxError) as e:
            cvx.cvx_render_noalloc(sess.ctx, cvx.make_views(too_many[:2]), out.data_ptr(),
                                   cvx.make_opts(**bad))
        assert e.value.code == cvx.CVX_ERR_INVALID_ARG
    # the largest allowed view set renders as cvx_render does
    most = too_many[:cvx.CVX_NOALLOC_MAX_VIEWS]
    ref, img, _, _ = _both(sess, most)
    np.testing.assert_array_equal(img, ref)

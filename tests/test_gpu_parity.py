"""GPU parity: the C-ABI HIP path against the CPU FP64 oracle on seeded inputs.

Bars (see the tolerance notes next to each check):
  * leaf sequences: bit-exact node ids and counts for every ray the oracle
    does not flag (within 1e-12 of a face of a visited leaf, or an ambiguous
    stop), for FP32_REBASED and FP64_PLAIN;
  * RGBA: <= 1e-3 absolute for the FP32 variants (FP16/RGBA8 leaves, FP32
    accumulators); FP64_PLAIN against the oracle within a bound derived from
    FP64 rounding of canvas-global parameters (see tol64);
  * FP32_NAIVE has no bar: its mismatch count is the expected failure.
"""
import math

import numpy as np
import pytest

from canvasgen import LEAF_F64, LEAF_RGBA8_F16, make_view, stereo_pair
from canvasgen import configs, trees
from oracle import oracle

from gpu_common import (all_ray_ids, compare_traces, merge_piece_traces, rgba_err,
                        sample_ray_ids)

pytestmark = pytest.mark.gpu

RGBA_TOL32 = 1e-3


def tol64(depth):
    # canvas-global FP64: t carries ~4 ulp of |t| <= 4 root edges, so a local
    # length l = dt * 2^depth differs by <= 2^-49 * 2^depth between two FP64
    # evaluations; with optical depth kappa <= 64 per leaf edge this bounds
    # the transmittance difference.
    return max(1e-11, 64.0 * 2.0 ** (depth - 49))


@pytest.fixture(scope="module")
def sess():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1704_02724_amd.session import Session
    s = Session(0)
    yield s
    s.close()


def _views_around(rng, n, W, H, inside=True, R=1.0):
    vs, off = [], 0
    for _ in range(n):
        e = rng.uniform(0.05 * R, 0.95 * R, 3) if inside else rng.uniform(-1.0, 2.0, 3) * R
        tgt = rng.uniform(0.2 * R, 0.8 * R, 3)
        vs.append(make_view(e, tgt - e, rng.uniform(0.3, 1.2), W, H, out_offset_px=off))
        off += W * H
    return vs


def _check(sess, canvases, views, variant, max_leaves=512, rgba_tol=RGBA_TOL32, out64=False,
           min_checked=0.9):
    for i, c in enumerate(canvases):
        sess.upload(i, c)
    ids = all_ray_ids(views)
    orc = oracle.render(canvases, views, ids, max_leaves=max_leaves)
    gpu = sess.trace(views, ids, max_leaves, variant, len64=out64)
    assert np.all((gpu["flags"] & 0x5) == 0), "step cap or broken link on a valid pool"
    cmp = compare_traces(orc, gpu, max_leaves)
    ok = cmp["ok_mask"]
    assert ok.mean() >= min_checked, cmp
    img = sess.render(views, variant, out_f64=out64).cpu().numpy()
    pix = np.concatenate([v["out_offset_px"] + np.arange(v["W"] * v["H"]) for v in views])
    err = rgba_err(img[pix], orc["rgba"], ok)
    # trace mode and render mode run the same per-ray code
    if not out64:
        np.testing.assert_array_equal(gpu["rgba"], img[pix].astype(np.float32))
    return cmp, err


@pytest.mark.parametrize("R,depth,seed", [(1, 5, 1), (2, 4, 2), (3, 4, 3), (1, 8, 4)])
def test_random_trees_fp64_plain(sess, R, depth, seed):
    cv = trees.random_tree(R, depth, seed=seed, p_split=0.5, max_nodes=8000, leaf_format=LEAF_F64)
    rng = np.random.Generator(np.random.PCG64(seed))
    views = _views_around(rng, 3, 24, 20, inside=True, R=1.0) + \
        [make_view((-0.6, 0.4, 1.7), (1.0, 0.1, -1.0), 0.8, 17, 31, out_offset_px=3 * 480)]
    cmp, err = _check(sess, [cv], views, "fp64_plain", out64=True)
    assert cmp["seq_mismatch"] == 0, cmp
    assert err <= tol64(depth), err


@pytest.mark.parametrize("R,depth,seed", [(1, 5, 11), (2, 5, 12), (1, 9, 13)])
def test_random_trees_fp32_rebased(sess, R, depth, seed):
    cv = trees.random_tree(R, depth, seed=seed, p_split=0.5, max_nodes=8000,
                           leaf_format=LEAF_RGBA8_F16, kappa_range=(0.0, 8.0))
    rng = np.random.Generator(np.random.PCG64(seed))
    views = _views_around(rng, 4, 23, 19, inside=seed % 2 == 0)
    cmp, err = _check(sess, [cv], views, "fp32_rebased")
    assert cmp["seq_mismatch"] == 0, cmp
    assert cmp["len_bad"] == 0, cmp
    assert err <= RGBA_TOL32, err


@pytest.mark.parametrize("depth", [16, 24, 30])
def test_deep_paths(sess, depth):
    """Long same-depth runs next to abrupt jumps of up to `depth` levels."""
    t = np.array([0.3 + 1 / 3000, 0.6 - 1 / 7000, 0.45 + 1 / 5000])
    cv = trees.deep_path_tree(depth, target=t, seed=depth, leaf_format=LEAF_RGBA8_F16, halo=2,
                              kappa_range=(0.0, 3.0))
    h = 2.0 ** -depth
    views = [
        make_view(t + h * np.array([-6.3, 0.37, 0.71]), (1.0, 0.05, -0.02), 0.7, 31, 29),
        make_view(t + h * np.array([0.2, 0.1, -0.3]), (0.3, -0.8, 0.5), 1.5, 27, 25,
                  out_offset_px=31 * 29),
        make_view((-0.5, 0.55, 0.2), t - np.array([-0.5, 0.55, 0.2]), 3 * h, 25, 21,
                  out_offset_px=31 * 29 + 27 * 25),
    ]
    cmp, err = _check(sess, [cv], views, "fp32_rebased")
    assert cmp["seq_mismatch"] == 0, cmp
    assert err <= RGBA_TOL32, err
    cmp64, err64 = _check(sess, [cv], views, "fp64_plain")
    assert cmp64["seq_mismatch"] == 0, cmp64
    assert err64 <= RGBA_TOL32, err64
    naive, _ = _check(sess, [cv], views, "fp32_naive", min_checked=0.0)
    print(f"depth {depth}: naive FP32 sequence mismatches {naive['seq_mismatch']} of {naive['n']}")


def test_tiny_config_fp64_everywhere(sess):
    w = configs.tiny(leaf_format=LEAF_F64)
    cmp, err = _check(sess, w.canvases, w.views, "fp64_plain", max_leaves=128, out64=True)
    assert cmp["seq_mismatch"] == 0, cmp
    assert err <= tol64(12), err
    print(f"tiny fp64: flagged {cmp['flagged']} of {cmp['n']}, max rgba err {err:.3g}")


def test_tiny_config_fp32(sess):
    w = configs.tiny(leaf_format=LEAF_RGBA8_F16)
    cmp, err = _check(sess, w.canvases, w.views, "fp32_rebased", max_leaves=128)
    assert cmp["seq_mismatch"] == 0, cmp
    assert err <= RGBA_TOL32, err
    naive, nerr = _check(sess, w.canvases, w.views, "fp32_naive", max_leaves=128, min_checked=0.0)
    print(f"tiny fp32: flagged {cmp['flagged']}, rgba err {err:.3g}; naive mismatches "
          f"{naive['seq_mismatch']}, naive rgba err {nerr:.3g}")


def test_determinism_across_tuning(sess):
    w = configs.tiny(leaf_format=LEAF_RGBA8_F16, W=101, H=77)
    sess.upload(0, w.canvases[0])
    ref = sess.render(w.views, "fp32_rebased").cpu().numpy()
    for tile, wgs, wg, top, sq in [((16, 4), 1, 64, 0, 0), ((64, 1), 7, 128, 1, 1),
                                   ((4, 16), 0, 256, 1, 0), ((32, 2), 3, 256, 0, 1),
                                   ((8, 8), 13, 64, 0, 0)]:
        img = sess.render(w.views, "fp32_rebased", tile=tile, workgroups=wgs, wg_size=wg,
                          top_lookup=top, single_queue=sq)
        np.testing.assert_array_equal(img.cpu().numpy(), ref)


@pytest.mark.parametrize("R,depth,seed", [(1, 9, 61), (2, 7, 62), (3, 6, 63)])
def test_top_table_matches_root_descent(sess, R, depth, seed):
    """Ray starts located through the top-level table or from the root array
    give the same images and the same leaf sequences."""
    cv = trees.random_tree(R, depth, seed=seed, max_nodes=40000, leaf_format=LEAF_RGBA8_F16)
    rng = np.random.Generator(np.random.PCG64(seed))
    views = _views_around(rng, 3, 40, 24, inside=True)
    sess.upload(0, cv)
    for var in ("fp32_rebased", "fp64_plain"):
        a = sess.render(views, var, top_lookup=0).cpu().numpy()
        b = sess.render(views, var, top_lookup=1).cpu().numpy()
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("R,depth,seed", [(1, 9, 64), (2, 7, 65), (3, 6, 66)])
def test_shared_eye_leaf_matches_per_ray_start(sess, R, depth, seed):
    """Views whose eye lies inside the canvas share the eye's leaf as the first
    leaf of every ray; the images equal those of per-ray starts, also for eyes
    on a cell plane (no sharing), on the canvas boundary and outside, and in
    a graph replayed with fewer views."""
    cv = trees.random_tree(R, depth, seed=seed, max_nodes=40000, leaf_format=LEAF_RGBA8_F16)
    rng = np.random.Generator(np.random.PCG64(seed))
    views = _views_around(rng, 3, 40, 24, inside=True, R=R)
    off = 3 * 40 * 24
    tgt = np.array([0.5, 0.5, 0.5]) * R
    for e in ([0.5 * R, 0.3 * R, 0.7 * R],            # on a plane of every depth
              [0.0, 0.41 * R, 0.37 * R],              # on the canvas boundary
              [-0.3 * R, 1.2 * R, 0.4 * R]):          # outside
        e = np.array(e)
        views.append(make_view(e, tgt - e, 0.8, 40, 24, out_offset_px=off))
        off += 40 * 24
    sess.upload(0, cv)
    for var in ("fp32_rebased", "fp64_plain", "fp32_cell_local"):
        a = sess.render(views, var, per_ray_start=0).cpu().numpy()
        b = sess.render(views, var, per_ray_start=1).cpu().numpy()
        np.testing.assert_array_equal(a, b)
    torch = sess.torch
    out = torch.full((off, 4), -1.0, dtype=torch.float32, device=sess.device)
    sess.render(views, "fp32_rebased", out=out, use_graph=True)
    full = out.cpu().numpy()
    out.fill_(-1.0)
    sess.render(views[:2], "fp32_rebased", out=out, use_graph=True)   # same graph, 2 views
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    np.testing.assert_array_equal(got[:2 * 40 * 24], full[:2 * 40 * 24])
    assert np.all(got[2 * 40 * 24:] == -1.0)


def test_graph_replay_matches_eager(sess):
    torch = sess.torch
    w = configs.tiny(leaf_format=LEAF_RGBA8_F16, W=64, H=48)
    sess.upload(0, w.canvases[0])
    v2 = [dict(w.views[0], eye=(0.45, 0.52, -0.6))]
    eager1 = sess.render(w.views, "fp32_rebased").cpu().numpy()
    eager2 = sess.render(v2, "fp32_rebased").cpu().numpy()
    out = torch.empty((64 * 48, 4), dtype=torch.float32, device=sess.device)
    for i in range(4):
        vs, ref = (w.views, eager1) if i % 2 == 0 else (v2, eager2)
        out.fill_(-1.0)
        sess.render(vs, "fp32_rebased", out=out, use_graph=True)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(out.cpu().numpy(), ref)
        _ = (torch.ones(1000, device=sess.device) * 2).sum().item()  # eager work in between


def test_multi_canvas_offsets_ragged(sess):
    a = trees.random_tree(1, 6, seed=21, max_nodes=6000, leaf_format=LEAF_RGBA8_F16)
    b = trees.random_tree(2, 5, seed=22, max_nodes=6000, leaf_format=LEAF_RGBA8_F16)
    views = [make_view((0.5, 0.5, -1.0), (0.01, 0.02, 1.0), 0.6, 37, 23, canvas_id=0),
             make_view((0.3, 0.2, 0.4), (0.5, 0.2, 0.3), 1.0, 1, 1, canvas_id=1,
                       out_offset_px=2000),
             make_view((1.5, 0.5, 0.5), (-1.0, 0.1, 0.05), 0.9, 64, 9, canvas_id=0,
                       out_offset_px=37 * 23)]
    cmp, err = _check(sess, [a, b], views, "fp32_rebased")
    assert cmp["seq_mismatch"] == 0 and err <= RGBA_TOL32, (cmp, err)


def test_alpha_stop(sess):
    cv = trees.random_tree(1, 6, seed=31, max_nodes=8000, leaf_format=LEAF_RGBA8_F16,
                           kappa_range=(0.5, 4.0))
    rng = np.random.Generator(np.random.PCG64(31))
    views = _views_around(rng, 2, 20, 20, inside=False)
    for v in views:
        v["alpha_stop"] = 0.9
    cmp, err = _check(sess, [cv], views, "fp32_rebased")
    assert cmp["seq_mismatch"] == 0 and err <= RGBA_TOL32, (cmp, err)
    cmp64, err64 = _check(sess, [cv], views, "fp64_plain")
    assert cmp64["seq_mismatch"] == 0, cmp64


def test_miss_gives_zero(sess):
    cv = trees.uniform_tree(1, 2, seed=1, leaf_format=LEAF_RGBA8_F16)
    sess.upload(0, cv)
    v = [make_view((-1.0, 0.5, 0.5), (-1.0, 0.0, 0.0), 0.5, 8, 8)]
    for var in ("fp32_rebased", "fp64_plain", "fp32_naive"):
        img = sess.render(v, var).cpu().numpy()
        assert np.all(img == 0.0)


def test_stats_match_oracle_counts(sess):
    cv = trees.random_tree(1, 7, seed=41, max_nodes=8000, leaf_format=LEAF_RGBA8_F16)
    rng = np.random.Generator(np.random.PCG64(41))
    views = _views_around(rng, 2, 32, 32, inside=True)
    sess.upload(0, cv)
    orc = oracle.render([cv], views)
    if np.any(orc["flags"]):
        pytest.skip("seeded views hit a flagged ray")
    for var in ("fp32_rebased", "fp64_plain"):
        st = sess.new_stats()
        sess.render(views, var, stats=st)
        s = st.cpu().numpy()
        assert s[0] == 2 * 32 * 32
        assert s[1] == orc["n_leaves"].sum()
        links = (orc["alg_bytes"] - 16 - 8 * orc["n_leaves"].astype(np.float64)) / 4
        assert s[2] + s[3] == links.sum()
        # loop iterations cover every leaf; lane slots are whole 64-lane tiles
        assert s[6] >= s[1] and s[7] >= s[6] and s[7] % 64 == 0


def test_error_paths(sess):
    from paper_1704_02724_amd import cvx
    cv = trees.random_tree(1, 4, seed=51, leaf_format=LEAF_RGBA8_F16)
    sess.upload(5, cv)
    v = [make_view((0.5, 0.5, -1.0), (0.0, 0.0, 1.0), 0.5, 8, 8, canvas_id=5)]
    ref = sess.render(v).cpu().numpy()
    bad = trees.random_tree(1, 4, seed=51, leaf_format=LEAF_RGBA8_F16)
    bad.nodes[int(bad.nodes[0, 0]) + 3, 1] = 7  # wrong parent
    with pytest.raises(cvx.CvxError) as e:
        sess.upload(5, bad)
    assert e.value.code == cvx.CVX_ERR_BAD_POOL
    np.testing.assert_array_equal(sess.render(v).cpu().numpy(), ref)  # old pool intact
    with pytest.raises(cvx.CvxError) as e:
        sess.render([dict(v[0], canvas_id=9)])
    assert e.value.code == cvx.CVX_ERR_INVALID_ARG
    f64 = trees.random_tree(1, 4, seed=52, leaf_format=LEAF_F64)
    sess.upload(6, f64)
    with pytest.raises(cvx.CvxError) as e:
        sess.render([dict(v[0], canvas_id=6)], "fp32_rebased")
    assert e.value.code == cvx.CVX_ERR_INVALID_ARG
    sess.free(6)
    with pytest.raises(cvx.CvxError) as e:
        sess.free(6)
    assert e.value.code == cvx.CVX_ERR_NOT_FOUND


def test_upload_oom_keeps_the_old_pool(sess):
    """cvx_upload_pool checks the device room a pool needs before allocating
    anything: with the device nearly full it returns CVX_ERR_OOM and the
    pool already under that canvas id renders as before."""
    from paper_1704_02724_amd import cvx
    torch = sess.torch
    cv = trees.random_tree(1, 4, seed=51, leaf_format=LEAF_RGBA8_F16)
    sess.upload(5, cv)
    v = [make_view((0.5, 0.5, -1.0), (0.0, 0.0, 1.0), 0.5, 16, 16, canvas_id=5)]
    out = torch.zeros((256, 4), dtype=torch.float32, device=sess.device)
    ref = sess.render(v, out=out).cpu().numpy()
    big = configs.tiny(leaf_format=LEAF_RGBA8_F16, W=8, H=8).canvases[0]
    need = 40 * big.n_nodes + 8 * len(big.leaves)  # the upload's own estimate, roughly
    keep = (64 << 20) + need // 4                  # below need + the 64 MiB margin
    torch.cuda.synchronize()
    fill = []
    try:
        while True:
            free, _ = torch.cuda.mem_get_info(sess.device)
            if free <= keep + (2 << 20):
                break
            chunk = min(free - keep, 16 << 30)
            fill.append(torch.empty(chunk, dtype=torch.uint8, device=sess.device))
        with pytest.raises(cvx.CvxError) as e:
            sess.upload(5, big)
        assert e.value.code == cvx.CVX_ERR_OOM
        assert "device bytes" in str(e.value)
    finally:
        del fill
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    np.testing.assert_array_equal(sess.render(v, out=out).cpu().numpy(), ref)


def test_wide_offsets_same_image(sess):
    """Pools of at most 2^28 nodes are read with 32-bit offsets unless
    wide_offsets asks for the 64-bit addressing that larger pools take; the
    images are the same in every tuned launch shape."""
    w = configs.tiny(leaf_format=LEAF_RGBA8_F16, W=120, H=90)
    sess.upload(0, w.canvases[0])
    for kw in (dict(), dict(tile=(16, 4), wg_size=64, top_lookup=1),
               dict(tile=(4, 16), wg_size=128, single_queue=1, per_ray_start=1)):
        ref = sess.render(w.views, "fp32_rebased", **kw).cpu().numpy()
        img = sess.render(w.views, "fp32_rebased", wide_offsets=1, **kw).cpu().numpy()
        np.testing.assert_array_equal(img, ref)
        img = sess.render(w.views, "fp32_rebased", wide_offsets=1, use_graph=True, **kw)
        np.testing.assert_array_equal(img.cpu().numpy(), ref)


def test_cast_events_time_the_kernel(sess):
    """cast_events: the library records the caller's two events around the
    cast kernel of an eager render; the image is the one a render without
    them gives, the measured span is positive and no longer than the events
    the caller records around the whole call, and a graph render rejects
    them."""
    import ctypes

    from paper_1704_02724_amd import cvx
    torch = sess.torch
    w = configs.tiny(leaf_format=LEAF_RGBA8_F16, W=160, H=96)
    sess.upload(0, w.canvases[0])
    ref = sess.render(w.views, "fp32_rebased").cpu().numpy()
    k0, k1, c0, c1 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    for e in (k0, k1):
        e.record(sess.stream)
    pair = (ctypes.c_void_p * 2)(k0.cuda_event, k1.cuda_event)
    for _ in range(2):
        c0.record(sess.stream)
        img = sess.render(w.views, "fp32_rebased", cast_events=ctypes.addressof(pair))
        c1.record(sess.stream)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(img.cpu().numpy(), ref)
        kernel, call = k0.elapsed_time(k1), c0.elapsed_time(c1)
        assert 0.0 < kernel <= call
    with pytest.raises(cvx.CvxError) as e:
        sess.render(w.views, "fp32_rebased", use_graph=True, cast_events=ctypes.addressof(pair))
    assert e.value.code == cvx.CVX_ERR_INVALID_ARG


def test_lane_refill_same_image(sess):
    """Lane refill (rays_per_wave > 64: finished lanes take the next rays of a
    work item of several tiles once refill_min lanes wait) runs the same
    per-ray arithmetic, so images equal one ray per lane bit for bit: views
    of ragged sizes whose items end mid-view, eyes inside the canvas (shared
    first leaf) and outside (rays that miss), rays that stop at an opacity,
    two canvases, eager and graph launches."""
    from paper_1704_02724_amd import cvx
    cv0 = trees.random_tree(1, 9, seed=81, max_nodes=60000, leaf_format=LEAF_RGBA8_F16)
    cv1 = trees.random_tree(2, 6, seed=82, max_nodes=60000, leaf_format=LEAF_RGBA8_F16)
    sess.upload(0, cv0)
    sess.upload(1, cv1)
    rng = np.random.Generator(np.random.PCG64(83))
    views, off = [], 0
    for ci, W, H, inside, stop in [(0, 77, 53, True, 1.0), (1, 120, 41, True, 0.7),
                                   (0, 33, 90, False, 1.0), (1, 64, 64, False, 0.95),
                                   (0, 9, 7, True, 1.0)]:
        e = rng.uniform(0.1, 0.9, 3) if inside else rng.uniform(-1.0, 2.0, 3)
        tgt = rng.uniform(0.3, 0.7, 3)
        views.append(make_view(e, tgt - e, rng.uniform(0.4, 1.1), W, H, canvas_id=ci,
                               out_offset_px=off, alpha_stop=stop))
        off += W * H
    for tile in ((8, 8), (16, 4), (4, 16)):
        ref = sess.render(views, "fp32_rebased", tile=tile).cpu().numpy()
        assert (ref[:, 3] > 0).any() and (ref[:, 3] == 0).any()
        for rpw, mn in ((128, 32), (256, 1), (512, 48), (1024, 64), (192, 16)):
            kw = dict(tile=tile, rays_per_wave=rpw, refill_min=mn)
            np.testing.assert_array_equal(sess.render(views, "fp32_rebased", **kw).cpu().numpy(),
                                          ref)
            img = sess.render(views, "fp32_rebased", use_graph=True, wg_size=64, **kw)
            np.testing.assert_array_equal(img.cpu().numpy(), ref)
    for bad in (dict(rays_per_wave=100), dict(rays_per_wave=2048), dict(refill_min=65)):
        with pytest.raises(cvx.CvxError) as e:
            sess.render(views, "fp32_rebased", **bad)
        assert e.value.code == cvx.CVX_ERR_INVALID_ARG


@pytest.mark.parametrize("pieces", [2, 4, 8])
def test_chord_pieces(sess, pieces):
    """Chord pieces: each ray's canvas chord cut into equal parameter pieces
    traced as separate work items and merged front to back.  The merged
    leaf sequences (a leaf cut by a boundary counted once) equal the
    oracle's outside the face band; the images agree with the whole-chord
    render within FP32 rounding and with the oracle within 1e-3; views that
    stop at an opacity are rendered whole (bit for bit)."""
    R, depth = 2, 7
    cv = trees.random_tree(R, depth, seed=91, max_nodes=60000, leaf_format=LEAF_RGBA8_F16)
    sess.upload(0, cv)
    rng = np.random.Generator(np.random.PCG64(92))
    views = _views_around(rng, 3, 37, 29, inside=True, R=R) + _views_around(rng, 2, 31, 23,
                                                                           inside=False, R=R)
    off = 0
    for i, v in enumerate(views):
        v["out_offset_px"] = off
        off += v["W"] * v["H"]
    views[1]["alpha_stop"] = 0.8
    ML = 512
    ids = all_ray_ids(views)
    orc = oracle.render([cv], views, ids, max_leaves=ML)
    whole = sess.render(views, "fp32_rebased").cpu().numpy()
    # a split ray's lengths come from a second rebase at the cut, each within
    # the FP32 length guard: the images differ by about as much as each
    # differs from the oracle, so both are held to its bar
    for kw in (dict(), dict(use_graph=True, tile=(16, 4), wg_size=64)):
        img = sess.render(views, "fp32_rebased", chord_pieces=pieces, **kw).cpu().numpy()
        assert np.abs(img - whole).max() <= RGBA_TOL32
        stop = slice(views[1]["out_offset_px"], views[1]["out_offset_px"] + 37 * 29)
        np.testing.assert_array_equal(img[stop], whole[stop])
    gpu = merge_piece_traces(sess.trace(views, ids, ML, "fp32_rebased", chord_pieces=pieces),
                             len(ids), pieces, ML)
    assert np.all((gpu["flags"] & 0x5) == 0)
    cmp = compare_traces(orc, gpu, ML)
    assert cmp["seq_mismatch"] == 0, cmp
    assert cmp["n"] - cmp["flagged"] >= 0.9 * cmp["n"]
    pix = np.concatenate([v["out_offset_px"] + np.arange(v["W"] * v["H"]) for v in views])
    assert rgba_err(img[pix], orc["rgba"], cmp["ok_mask"]) <= RGBA_TOL32
    assert np.abs(gpu["rgba"] - img[pix]).max() <= 1e-6
    from paper_1704_02724_amd import cvx
    for bad in (dict(chord_pieces=3), dict(chord_pieces=2, rays_per_wave=128)):
        with pytest.raises(cvx.CvxError) as e:
            sess.render(views, "fp32_rebased", **bad)
        assert e.value.code == cvx.CVX_ERR_INVALID_ARG
    with pytest.raises(cvx.CvxError) as e:
        sess.render(views, "fp64_plain", chord_pieces=2)
    assert e.value.code == cvx.CVX_ERR_INVALID_ARG


def test_autotune_picks_a_timed_shape_and_keeps_the_image(sess):
    """cvx_autotune times every candidate launch shape; every candidate renders
    the same image, and the one it returns is the fastest it timed."""
    from paper_1704_02724_amd import cvx
    w = configs.tiny(leaf_format=LEAF_RGBA8_F16, W=96, H=80)
    sess.upload(0, w.canvases[0])
    ref = sess.render(w.views, "fp32_rebased").cpu().numpy()
    out = sess.torch.full((96 * 80, 4), -1.0, dtype=sess.torch.float32, device=sess.device)
    tuning, rows = sess.autotune(w.views, "fp32_rebased", out=out, reps=2)
    sess.torch.cuda.synchronize()
    # the last candidate timed splits chords: the same image within the bar
    assert np.abs(out.cpu().numpy() - ref).max() <= RGBA_TOL32
    assert len(rows) == 2 * 2 * 4 * 3 * 4 + 6 + 3
    assert {(r[0], r[1]) for r in rows} == {(8, 8), (16, 4), (4, 16), (32, 2)}
    assert {r[5] for r in rows} == {0, 1} and {r[6] for r in rows} == {0, 1}
    assert all(r[4] > 0.0 for r in rows)
    # lane refill is timed on the fastest one-ray-per-lane shape
    plain = [r for r in rows if r[7] == 64 and r[9] == 1]
    refill = [r for r in rows if r[7] > 64]
    split = [r for r in rows if r[9] > 1]
    assert len(plain) == 192 and all(r[8] == 0 for r in plain)
    shape = min(plain, key=lambda r: r[4])
    assert {(r[7], r[8]) for r in refill} == {(a, b) for a in (128, 256) for b in (16, 32, 48)}
    assert sorted(r[9] for r in split) == [2, 4, 8] and all(r[7] == 64 for r in split)
    assert all(r[:4] == shape[:4] and r[5:7] == shape[5:7] for r in refill + split)
    best = min(rows, key=lambda r: r[4])
    assert tuning == dict(tile=(best[0], best[1]), workgroups=best[3], wg_size=best[2],
                          top_lookup=best[5], single_queue=best[6], rays_per_wave=best[7],
                          refill_min=best[8], chord_pieces=best[9])
    img = sess.render(w.views, "fp32_rebased", use_graph=True, **tuning)
    if tuning["chord_pieces"] > 1:
        assert np.abs(img.cpu().numpy() - ref).max() <= RGBA_TOL32
    else:
        np.testing.assert_array_equal(img.cpu().numpy(), ref)
    varr = cvx.make_views(w.views)
    for reps, base in ((0, None), (2, cvx.make_opts("fp32_rebased", stats_ptr=sess.new_stats().data_ptr()))):
        with pytest.raises(cvx.CvxError) as e:
            cvx.cvx_autotune(sess.ctx, varr, out.data_ptr(), base, reps)
        assert e.value.code == cvx.CVX_ERR_INVALID_ARG

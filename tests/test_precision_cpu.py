"""CPU pins of the precision experiment's own FP64 arithmetic: its pixel
directions are the oracle's (same convention, same operation order) and its
canvas chords are the oracle's chords."""
import numpy as np

from canvasgen import LEAF_F64, make_view, trees
from oracle import oracle

from paper_1704_02724_amd import precision


def test_pixel_rays_and_chords_match_the_oracle():
    rng = np.random.Generator(np.random.PCG64(91))
    cv = trees.random_tree(1, 3, seed=91, leaf_format=LEAF_F64)
    for _ in range(4):
        e = rng.uniform(-0.5, 1.5, 3)
        v = make_view(e, rng.uniform(0.2, 0.8, 3) - e, rng.uniform(0.3, 1.2), 17, 11)
        px = np.arange(17 * 11, dtype=np.int64)
        d = precision.pixel_rays(v, px)
        for i in rng.choice(len(px), 20, replace=False):
            ref = oracle.ray_dir(v, int(px[i] % 17), int(px[i] // 17))
            np.testing.assert_allclose(d[i], ref, rtol=0, atol=4e-16)
        o = np.asarray(v["eye"], np.float64)
        t0, t1 = precision.canvas_chord(o, d, 1.0)
        orc = oracle.render([cv], [v])
        hit = t1 > t0
        np.testing.assert_array_equal(hit, orc["chord"] > 0)
        np.testing.assert_allclose((t1 - t0)[hit], orc["chord"][hit], rtol=1e-13, atol=1e-15)

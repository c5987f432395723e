"""CPU checks of the precision experiment's exact rays: they are the
oracle's own ray set-up (oracle.ray_setup), which must agree with the
oracle's per-pixel direction and with the chord its traversal covers, and
give the closed-form chord of axis-aligned rays through the canvas."""
import numpy as np

from canvasgen import LEAF_F64, make_view, trees
from oracle import oracle


def test_ray_setup_is_the_oracles_ray():
    rng = np.random.Generator(np.random.PCG64(91))
    cv = trees.random_tree(1, 3, seed=91, leaf_format=LEAF_F64)
    for _ in range(4):
        e = rng.uniform(-0.5, 1.5, 3)
        v = make_view(e, rng.uniform(0.2, 0.8, 3) - e, rng.uniform(0.3, 1.2), 17, 11)
        px = np.arange(17 * 11, dtype=np.int64)
        d, t0, t1 = oracle.ray_setup(cv, v, px)
        for i in rng.choice(len(px), 20, replace=False):
            np.testing.assert_array_equal(d[i], oracle.ray_dir(v, int(px[i] % 17),
                                                               int(px[i] // 17)))
        orc = oracle.render([cv], [v])
        hit = t1 > t0
        np.testing.assert_array_equal(hit, orc["chord"] > 0)
        np.testing.assert_array_equal((t1 - t0)[hit], orc["chord"][hit])
        # the traversal's segments add up to the same chord
        np.testing.assert_allclose(orc["sum_len"][hit], (t1 - t0)[hit], rtol=0, atol=1e-13)


def test_ray_setup_axis_aligned_chords():
    """A ray along +z from z = -0.5 through the unit canvas enters at t = 0.5
    and leaves at 1.5; from the inside (z = 0.25) it starts at t = 0."""
    cv = trees.random_tree(1, 2, seed=3, leaf_format=LEAF_F64)
    for z, want in ((-0.5, (0.5, 1.5)), (0.25, (0.0, 0.75))):
        v = make_view((0.3, 0.6, z), (0.0, 0.0, 1.0), 1e-9, 1, 1)
        d, t0, t1 = oracle.ray_setup(cv, v, np.array([0]))
        assert abs(d[0, 2] - 1.0) < 1e-15 and abs(d[0, 0]) < 1e-8 and abs(d[0, 1]) < 1e-8
        assert abs(t0[0] - want[0]) < 1e-12 and abs(t1[0] - want[1]) < 1e-12
    v = make_view((2.0, 2.0, 2.0), (1.0, 0.0, 0.0), 0.1, 1, 1)  # outside, looking away
    _, t0, t1 = oracle.ray_setup(cv, v, np.array([0]))
    assert t0[0] == 0.0 and t1[0] == 0.0

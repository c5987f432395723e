"""Shared test helpers: rays expressed as 1x1 views."""
import numpy as np

from canvasgen import make_view


def ray_views(eyes, dirs, canvas_id=0, alpha_stop=1.0):
    """One 1x1 view per ray: its single pixel looks exactly along fwd."""
    out = []
    for e, d in zip(eyes, dirs):
        out.append(make_view(e, d, 1.0, 1, 1, canvas_id=canvas_id, alpha_stop=alpha_stop))
    return out


def random_rays(rng, n, inside_frac=0.5, R=1.0):
    eyes, dirs = [], []
    for _ in range(n):
        if rng.uniform() < inside_frac:
            e = rng.uniform(0.0, R, 3)
        else:
            e = rng.uniform(-1.0 * R, 2.0 * R, 3)
        tgt = rng.uniform(0.0, R, 3)
        d = tgt - e
        if np.linalg.norm(d) < 1e-6:
            d = rng.normal(size=3)
        eyes.append(e)
        dirs.append(d / np.linalg.norm(d))
    return eyes, dirs

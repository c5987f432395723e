"""Seeded synthetic brush strokes (input generation only).

The paper's paintings are not available, so seeded strokes stand in for them.
A stroke follows the painting model of Sec. 5.1: a path sampled into spherical
stamps of one radius, one brush colour and one opacity density.  The recipe:

* radius r: log2(r) uniform in [lg_lo, lg_hi];
* brush colour: RGB uniform in [0, 1]^3, quantised to k/255;
* opacity density sigma: uniform in [1, 50] (per stroke radius);
* path: a cubic Bezier curve; P0 uniform in the placement box and each next
  control point P_{j+1} = P_j + 12 r u_j with u_j a uniform random unit vector;
* stamps: spheres of radius r centred on the curve at arc lengths i*r/2 for
  i = 0..63 (stamps past the end of the curve are dropped).

Every number is drawn from ``numpy.random.Generator(PCG64(seed))`` in the
order: radii, colours, densities, start points, directions.
"""
from __future__ import annotations

import numpy as np

N_STAMPS = 64
N_CURVE_SAMPLES = 1024


class StrokeSet:
    """Flat arrays describing a batch of strokes."""

    def __init__(self, radius, rgb, sigma, stamp_off, stamps):
        self.radius = np.ascontiguousarray(radius, dtype=np.float64)
        self.rgb = np.ascontiguousarray(rgb, dtype=np.float64)
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        self.stamp_off = np.ascontiguousarray(stamp_off, dtype=np.int64)
        self.stamps = np.ascontiguousarray(stamps, dtype=np.float64)  # (n_stamps, 4): x y z r

    @property
    def n(self):
        return len(self.radius)

    def stamps_of(self, i):
        return self.stamps[self.stamp_off[i]:self.stamp_off[i + 1]]

    @staticmethod
    def concat(sets):
        offs, acc = [np.zeros(1, np.int64)], 0
        for s in sets:
            offs.append(s.stamp_off[1:] + acc)
            acc += len(s.stamps)
        return StrokeSet(np.concatenate([s.radius for s in sets]),
                         np.concatenate([s.rgb for s in sets]),
                         np.concatenate([s.sigma for s in sets]),
                         np.concatenate(offs),
                         np.concatenate([s.stamps for s in sets]) if sets else np.zeros((0, 4)))


def _bezier(ctrl, ts):
    """ctrl (n,4,3), ts (m,) -> (n,m,3)."""
    u = 1.0 - ts
    b = np.stack([u ** 3, 3 * u * u * ts, 3 * u * ts * ts, ts ** 3], axis=0)  # (4,m)
    return np.einsum("km,nkd->nmd", b, ctrl)


def gen_strokes(rng: np.random.Generator, n: int, lg_lo: float, lg_hi: float,
                box_lo=(0.0, 0.0, 0.0), box_size=1.0) -> StrokeSet:
    radius = 2.0 ** rng.uniform(lg_lo, lg_hi, n)
    rgb = np.round(rng.uniform(0.0, 1.0, (n, 3)) * 255.0) / 255.0
    sigma = rng.uniform(1.0, 50.0, n)
    p0 = np.asarray(box_lo, np.float64)[None, :] + rng.uniform(0.0, 1.0, (n, 3)) * box_size
    u = rng.normal(size=(n, 3, 3))
    u /= np.linalg.norm(u, axis=2, keepdims=True)
    steps = 12.0 * radius[:, None, None] * u
    ctrl = np.concatenate([p0[:, None, :], p0[:, None, :] + np.cumsum(steps, axis=1)], axis=1)

    ts = np.linspace(0.0, 1.0, N_CURVE_SAMPLES + 1)
    offs = [0]
    stamps = []
    chunk = 2048
    for c0 in range(0, n, chunk):
        pts = _bezier(ctrl[c0:c0 + chunk], ts)                      # (c,m,3)
        seg = np.linalg.norm(np.diff(pts, axis=1), axis=2)          # (c,m-1)
        arc = np.concatenate([np.zeros((len(pts), 1)), np.cumsum(seg, axis=1)], axis=1)
        for j in range(len(pts)):
            r = radius[c0 + j]
            want = np.arange(N_STAMPS) * (0.5 * r)
            want = want[want <= arc[j, -1]]
            pos = np.stack([np.interp(want, arc[j], pts[j, :, a]) for a in range(3)], axis=1)
            st = np.empty((len(want), 4))
            st[:, :3] = pos
            st[:, 3] = r
            stamps.append(st)
            offs.append(offs[-1] + len(want))
    return StrokeSet(radius, rgb, sigma, np.asarray(offs, np.int64),
                     np.concatenate(stamps) if stamps else np.zeros((0, 4)))

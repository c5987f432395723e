"""The precision experiment of Sec. 6.3: per-pixel ray-angle error, cells
crossed and error against ray length, for each traversal variant.

Test infrastructure (the analysis of trace-mode output; the library does not
use it).  For every pixel the caster reports (trace mode) the exit point of
the last leaf as the variant computed it.  The exact ray is the oracle's
FP64 ray of that pixel (its direction and canvas chord, oracle.ray_setup);
the angle error is the angle between (end point - eye) and that direction,
the along-ray error the difference between the end point's distance along it
and the exact canvas exit, over the chord length L.  The paper's stated
worst case for its cell-local scheme is an angle of
asin(sqrt(2) (e0 / L + 7.5 eps)) with eps = 2^-23 (e0 = start-point error);
for the half-precision traversal eps = 2^-10.

    python tests/precision_experiment.py --workload depth24
prints one JSON summary (binned by L and by cells crossed).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import oracle  # noqa: E402

EPS32 = 2.0 ** -23
EPS16 = 2.0 ** -10


def paper_bound_deg(eps):
    """The worst-case ray angle of Sec. 6.3 with no start-point error."""
    return math.degrees(math.asin(math.sqrt(2) * 7.5 * eps))


def measure(sess, canvases, views, variant, max_rays=None, seed=0):
    """Per-pixel errors of one variant over all (or max_rays sampled) pixels."""
    rows = []
    rng = np.random.Generator(np.random.PCG64(seed))
    for vi, v in enumerate(views):
        n = v["W"] * v["H"]
        px = np.arange(n, dtype=np.int64)
        if max_rays and n > max_rays // len(views):
            px = np.sort(rng.choice(n, max_rays // len(views), replace=False))
        cv = canvases[v["canvas_id"]]
        o = (np.asarray(v["eye"], np.float64) - np.asarray(cv.origin)) / cv.root_edge
        d, t0, t1 = oracle.ray_setup(cv, v, px)
        ids = (np.uint64(vi) << np.uint64(32)) | px.astype(np.uint64)
        tr = sess.trace(views, ids, 1, variant, end_point=True)
        e = tr["end_point"] - o[None, :]
        along = (e * d).sum(1)
        cross = np.cross(e, d)
        sin_t = np.sqrt((cross * cross).sum(1)) / np.maximum(np.sqrt((e * e).sum(1)), 1e-300)
        hit = (t1 > t0) & (tr["n_leaves"] > 0) & (v["alpha_stop"] >= 1.0)
        L = t1 - t0
        rows.append(dict(angle_deg=np.degrees(np.arcsin(np.minimum(sin_t, 1.0)))[hit],
                         along_rel=(np.abs(along - t1) / np.maximum(L, 1e-300))[hit],
                         L=L[hit], cells=tr["n_leaves"][hit].astype(np.int64)))
    return {k: np.concatenate([r[k] for r in rows]) for k in rows[0]}


def _bins(x, y, edges):
    out = []
    for a, b in zip(edges[:-1], edges[1:]):
        m = (x >= a) & (x < b)
        if m.sum() == 0:
            continue
        out.append(dict(lo=float(a), hi=float(b), rays=int(m.sum()),
                        median=float(np.median(y[m])), p99=float(np.quantile(y[m], 0.99)),
                        max=float(y[m].max())))
    return out


def summarise(m):
    a = m["angle_deg"]
    L = m["L"]
    Le = np.quantile(L, np.linspace(0, 1, 9))
    Le[-1] = np.nextafter(Le[-1], np.inf)
    ce = np.unique(np.quantile(m["cells"], np.linspace(0, 1, 9)).astype(np.int64))
    ce[-1] += 1
    return dict(rays=int(len(a)), angle_deg=dict(median=float(np.median(a)),
                                                 p99=float(np.quantile(a, 0.99)), max=float(a.max())),
                along_rel=dict(median=float(np.median(m["along_rel"])),
                               max=float(m["along_rel"].max())),
                by_length=_bins(L, a, Le), by_cells=_bins(m["cells"], a, ce),
                paper_bound_deg_at_e0_0=dict(fp32=paper_bound_deg(EPS32),
                                             fp16=paper_bound_deg(EPS16)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="depth24")
    ap.add_argument("--variants", default="fp16_cell_local,fp32_cell_local,fp32_naive,fp32_rebased,fp64_plain")
    ap.add_argument("--max-rays", type=int, default=0)
    args = ap.parse_args()
    from canvasgen import configs
    from paper_1704_02724_amd.session import Session
    w = {"depth24": configs.depth24, "depth30": configs.depth30}[args.workload]()
    sess = Session(0)
    for i, c in enumerate(w.canvases):
        sess.upload(i, c)
    res = dict(workload=args.workload, rays=w.n_rays, variants={})
    for var in args.variants.split(","):
        res["variants"][var] = summarise(measure(sess, w.canvases, w.views, var,
                                                 args.max_rays or None))
        print(f"{var}: {res['variants'][var]['angle_deg']}", file=sys.stderr, flush=True)
    sess.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

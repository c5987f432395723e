"""Helpers for the GPU parity tests: run the C-ABI path and the oracle on the
same seeded inputs and compare them ray by ray."""
from __future__ import annotations

import numpy as np

from oracle import oracle

ORC_SKIP = oracle.FLAG_NEAR_FACE | oracle.FLAG_TERM_AMBIG


def all_ray_ids(views):
    ids = []
    for i, v in enumerate(views):
        ids.append((np.uint64(i) << np.uint64(32)) | np.arange(v["W"] * v["H"], dtype=np.uint64))
    return np.concatenate(ids)


def sample_ray_ids(views, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.array([v["W"] * v["H"] for v in views], np.int64)
    vi = rng.choice(len(views), size=n, p=sizes / sizes.sum())
    px = (rng.uniform(0, 1, n) * sizes[vi]).astype(np.int64)
    ids = (vi.astype(np.uint64) << np.uint64(32)) | px.astype(np.uint64)
    return np.unique(ids)


def compare_traces(orc, gpu, max_leaves, len_atol=2e-4):
    """Compare oracle and GPU traces; returns a dict of counts.

    Rays the oracle flags (within 1e-12 of a face of a visited leaf, or with
    an ambiguous termination) are excluded from the sequence check."""
    n = len(orc["flags"])
    skip = (orc["flags"] & ORC_SKIP) != 0
    ok = ~skip
    cnt_eq = gpu["n_leaves"] == orc["n_leaves"]
    m = np.minimum(orc["n_leaves"], max_leaves).astype(np.int64)
    pos = np.arange(max_leaves)[None, :] < m[:, None]
    id_eq = np.all((gpu["leaf_ids"][:, :max_leaves] == orc["leaf_ids"]) | ~pos, axis=1)
    seq_ok = cnt_eq & id_eq
    len_err = np.where(pos & (seq_ok[:, None]), np.abs(gpu["local_len"][:, :max_leaves] -
                                                        orc["leaf_len"]), 0.0)
    return dict(n=n, flagged=int(skip.sum()), seq_mismatch=int((~seq_ok & ok).sum()),
                seq_mismatch_all=int((~seq_ok).sum()),
                max_len_err=float(len_err[ok].max()) if ok.any() else 0.0,
                len_bad=int((len_err[ok] > len_atol).sum()) if ok.any() else 0,
                ok_mask=ok, seq_ok=seq_ok)


def rgba_err(a, b, mask=None):
    e = np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)).max(axis=1)
    if mask is not None:
        e = e[mask]
    return float(e.max()) if len(e) else 0.0


def merge_piece_traces(gpu, n, pieces, max_leaves):
    """Whole-ray traces from a chord-piece trace (rows (ray, piece), ray-major):
    the pieces' leaf sequences concatenated, a leaf cut by a piece boundary
    (the last of one piece and the first of the next) counted once; flags
    or-ed; RGBA merged front to back from the pieces' (colour, transmittance)."""
    ids = gpu["leaf_ids"].reshape(n, pieces, -1)
    cnt = gpu["n_leaves"].reshape(n, pieces).astype(np.int64)
    out_ids = np.zeros((n, max_leaves), np.uint32)
    out_n = np.zeros(n, np.uint32)
    for r in range(n):
        seq = []
        for j in range(pieces):
            part = ids[r, j, :min(int(cnt[r, j]), max_leaves)].tolist()
            if seq and part and part[0] == seq[-1]:
                part = part[1:]
            seq.extend(part)
        out_n[r] = len(seq)
        seq = seq[:max_leaves]
        out_ids[r, :len(seq)] = seq
    rgba = gpu["rgba"].reshape(n, pieces, 4).astype(np.float64)
    c = np.zeros((n, 3))
    t = np.ones(n)
    for j in range(pieces):
        c += t[:, None] * rgba[:, j, :3]
        t *= rgba[:, j, 3]
    return dict(leaf_ids=out_ids, n_leaves=out_n,
                flags=np.bitwise_or.reduce(gpu["flags"].reshape(n, pieces), axis=1),
                rgba=np.concatenate([c, (1.0 - t)[:, None]], axis=1),
                local_len=np.zeros((n, max_leaves), np.float32))

"""Benchmark: Mrays/s of the FP32-rebased deep-octree ray caster on one MI355X.

Headline workload (default "large"): a unit-cube canvas refined to depth 26
by 55,000 seeded strokes (radius 2^-24..2^-2, 1.46 G nodes, 35 GB of node
records and payloads in HBM), rendered as a stereo pair of 2160x2160 views
from an eye just outside a small stroke, rays stopping once their opacity
reaches 0.99.  One step = one cvx_render call over both views (a replayed HIP
graph, one persistent launch), with the pool already resident in HBM.

The line also carries, for the headline workload:
  * the FP64-plain GPU caster timed on the same views,
  * parity against the CPU FP64 oracle on a seeded ray sample (leaf
    sequences bit-exact outside 1e-12 face bands, RGBA <= 1e-3); `value` is
    null when parity fails,
  * the naive canvas-global FP32 caster on the same sample (its leaf-sequence
    mismatch rate and RGBA error: the precision failure the rebase removes),
  * the roofline of the cast kernel: the bound the committed rocprofv3
    counters show (vector instruction issue), the kernel's issue rate against
    the chip's, and its algorithmic and measured HBM bytes against 8 TB/s,
  * the CPU oracle timed on the host cores over a bounded seeded sample,
and under "configs" the same measurements (fewer steps, no CPU leg) for the
other workloads: the depth-24 stereo pair, the depth-30 zoomed view, the
batch of 64 views over 8 canvases, and the depth-24 and depth-30 canvases
refined with k = 10 (leaves of 10 per stroke radius instead of 4: 0.66 G and
0.18 G nodes, about 390 and 550 leaves per ray).
"""
from __future__ import annotations

import argparse
import ctypes
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # bytes/s, MI355X HBM3E
N_SIMD = 1024      # 256 compute units x 4 SIMDs
CLOCK = 2.4e9      # peak engine clock, Hz
# Peak wave64 vector-instruction issue per SIMD per cycle: a SIMD executes a
# 32-bit vector instruction of a wave64 over 64 lanes at 32 lanes per clock
# (the non-packed FP32 rate behind the 157.3 TFLOP/s peak: 256 CUs x 4 SIMDs
# x 32 lanes x 2 flops x 2.4 GHz), so at most one instruction every two
# clocks.
VALU_ISSUE_PER_SIMD_CYCLE = 0.5
VALU_PEAK = N_SIMD * CLOCK * VALU_ISSUE_PER_SIMD_CYCLE  # wave64 instructions/s

WORKLOADS = ("tiny", "depth24", "depth24_k10", "depth30", "depth30_k10", "batch", "large")
ML = 1024  # leaves recorded per ray in the parity traces


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of what the cast kernel is compiled from: its sources and the
    compiler flags."""
    import hashlib
    from paper_1704_02724_amd.build import HIPCC_FLAGS
    h = hashlib.sha256()
    for f in ("paper_1704_02724_amd/csrc/cvx_cast.hip", "paper_1704_02724_amd/csrc/cvx_internal.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(HIPCC_FLAGS).encode())
    return h.hexdigest()[:16]


def profiled_counts(variant, workload):
    """(HBM bytes, VALU wave-instructions) per launch from the committed
    rocprofv3 summary of this kernel and workload; (None, None) when the kernel
    source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"k_cast_{variant}_{workload}.md")
    if not os.path.exists(path):
        return None, None
    vals = {}
    for line in open(path):
        if line.startswith("| SQ_INSTS_VALU |"):
            vals["valu"] = line.split("|")[2].strip()
        elif ":" in line:
            k, _, v = line.partition(":")
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None, None
    out = []
    for k in ("traffic_bytes_per_launch", "valu"):
        try:
            out.append(float(vals[k]))
        except (KeyError, ValueError):
            out.append(None)
    return tuple(out)


def roofline(alg_bytes, kernel_s, traffic_b, valu_instr, copy_bps):
    """The roofline object of the cast kernel.

    The kernel has no contraction (no MFMA) and, by its counters, moves far
    fewer HBM bytes than it issues vector instructions for: the L2 serves
    most of the node loads.  Its bound is then vector issue ("alu"):
    achieved = wave64 VALU instructions per second (profiled count per launch
    over the kernel's mean duration, timed by an event pair that the library
    records around the kernel's own launch), peak = VALU_PEAK.  The HBM figures sit
    beside it: the algorithmic bytes (16 B per pixel + 8 B per leaf payload
    + 4 B per neighbour link or level descended, counted by the kernel) and
    the measured HBM bytes, each over 8 TB/s."""
    alg_bps = alg_bytes / kernel_s
    traffic_bps = traffic_b / kernel_s if traffic_b else None
    valu_rate = valu_instr / kernel_s if valu_instr else None
    issue_frac = valu_rate / VALU_PEAK if valu_rate else None
    hbm_frac = traffic_bps / HBM_PEAK if traffic_bps else None
    if issue_frac is not None and hbm_frac is not None:
        bound = "alu" if issue_frac >= hbm_frac else "hbm"
    else:
        bound = None  # the committed profile is of another build of the kernel
    r = {"bound": bound}
    if bound == "hbm":
        r.update(achieved=round(traffic_bps / 1e9, 1), peak=HBM_PEAK / 1e9, unit="GB/s",
                 frac=round(hbm_frac, 4))
    elif bound == "alu":
        r.update(achieved=round(valu_rate / 1e9, 1), peak=round(VALU_PEAK / 1e9, 1),
                 unit="G wave64 VALU instr/s", frac=round(issue_frac, 4))
    else:
        r.update(achieved=None, peak=None, unit=None, frac=None)
    r.update({
        # HBM bytes per second from the committed profile (FETCH_SIZE +
        # WRITE_SIZE, calibrated on a device copy)
        "traffic": round(traffic_bps / 1e9, 1) if traffic_bps else None,
        "traffic_unit": "GB/s",
        "traffic_bytes_per_launch": traffic_b,
        "hbm_measured_frac": round(hbm_frac, 4) if hbm_frac else None,
        "alg_bytes_per_launch": alg_bytes,
        "alg_GBps": round(alg_bps / 1e9, 1),
        "alg_bytes_frac": round(alg_bps / HBM_PEAK, 4),
        "kernel_ms": round(kernel_s * 1e3, 4),
        "measured_copy_GBps": round(copy_bps / 1e9, 1) if copy_bps else None,
        "alg_bytes_frac_of_measured_copy": round(alg_bps / copy_bps, 4) if copy_bps else None,
        "valu_wave_instr_per_launch": valu_instr,
        "valu_per_simd_cycle": round(valu_rate / (N_SIMD * CLOCK), 3) if valu_rate else None,
    })
    return r


def build_workload(name, threads):
    from canvasgen import configs
    if name == "depth24":
        return configs.depth24(threads=threads)
    if name == "depth24_k10":
        return configs.depth24(k=10.0, threads=threads)
    if name == "depth30":
        return configs.depth30(threads=threads)
    if name == "depth30_k10":
        return configs.depth30(k=10.0, threads=threads)
    if name == "tiny":
        from canvasgen import LEAF_RGBA8_F16
        return configs.tiny(leaf_format=LEAF_RGBA8_F16)
    if name == "batch":
        return configs.batch(threads=threads)
    if name == "large":
        return configs.large(threads=threads)
    raise SystemExit(f"unknown workload {name}")


def sample_ids(views, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.array([v["W"] * v["H"] for v in views], np.int64)
    vi = rng.choice(len(views), size=n, p=sizes / sizes.sum())
    px = (rng.uniform(0, 1, n) * sizes[vi]).astype(np.int64)
    return np.unique((vi.astype(np.uint64) << np.uint64(32)) | px.astype(np.uint64))


def time_variant(sess, views, variant, steps, warmup, tuning):
    torch = sess.torch
    out = torch.empty((sess.out_pixels(views), 4), dtype=torch.float32, device=sess.device)
    for _ in range(warmup):
        sess.render(views, variant, out=out, use_graph=True, **tuning)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(sess.stream)
        sess.render(views, variant, out=out, use_graph=True, **tuning)
        e.record(sess.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([s.elapsed_time(e) for s, e in ev])  # ms
    return out, wall, per


def time_cast_kernel(sess, views, variant, steps, tuning):
    """Durations (ms) of the cast kernel alone over `steps` eager renders:
    the library records a caller's event pair right before and right after
    the kernel's launch (cast_events), so the view staging and the shared
    first-leaf kernel that precede it in every call stay outside."""
    torch = sess.torch
    out = torch.empty((sess.out_pixels(views), 4), dtype=torch.float32, device=sess.device)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for s, e in ev:  # creates the events
        s.record(sess.stream)
        e.record(sess.stream)
    pairs = [(ctypes.c_void_p * 2)(s.cuda_event, e.cuda_event) for s, e in ev]
    sess.render(views, variant, out=out, use_graph=False, **tuning)
    torch.cuda.synchronize()
    for pr in pairs:
        sess.render(views, variant, out=out, use_graph=False, cast_events=ctypes.addressof(pr),
                    **tuning)
    torch.cuda.synchronize()
    return np.array([s.elapsed_time(e) for s, e in ev])


def time_per_view(sess, views, variant, steps, tuning):
    """The same views rendered with one cvx_render (one persistent launch) per
    view, each a replayed graph; returns wall seconds per step."""
    torch = sess.torch
    out = torch.empty((sess.out_pixels(views), 4), dtype=torch.float32, device=sess.device)
    for v in views:
        sess.render([v], variant, out=out, use_graph=True, **tuning)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for v in views:
            sess.render([v], variant, out=out, use_graph=True, **tuning)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def edit_bench(sess, cv, n_paint, n_refine, n_coarsen, seed):
    """Times cvx_edit_pool on a second copy of the canvas against a full
    cvx_upload_pool: two batches of paints, refinements and coarsenings on
    disjoint nodes, the first of which grows the pool (new capacity, the visit
    marks of the link rebuild) and the second of which refines into the groups
    the first one freed.  A single paint before them builds the host mirror."""
    from canvasgen.pool import LEAF, LEAF_DTYPE
    from paper_1704_02724_amd.cvx import EDIT_DTYPE
    torch = sess.torch
    rng = np.random.Generator(np.random.PCG64(seed))
    child = cv.nodes[:, 0]
    is_leaf = (child & LEAF) != 0
    internal = np.nonzero(~is_leaf)[0]
    kids = child[internal][:, None].astype(np.int64) + np.arange(8)[None, :]
    ok = np.all(is_leaf[kids], axis=1)
    coarse = rng.permutation(internal[ok])[:2 * n_coarsen]
    busy = np.zeros(len(child), bool)
    busy[(child[coarse][:, None].astype(np.int64) + np.arange(8)[None, :]).ravel()] = True
    # leaves in the tree: the padding slots after the roots have no parent
    in_tree = (cv.nodes[:, 1] != 0xFFFFFFFF) | (np.arange(len(child)) < cv.R ** 3)
    cand = np.nonzero(is_leaf & ~busy & in_tree)[0]
    pick = rng.permutation(cand)[:2 * (n_paint + n_refine) + 1]
    n_pay = n_paint + 8 * n_refine + n_coarsen
    pays = np.zeros(n_pay, LEAF_DTYPE[cv.leaf_format])
    if cv.leaf_format == 0:
        pays["r"], pays["g"], pays["b"] = (rng.integers(0, 256, (3, n_pay))).astype(np.uint8)
        pays["kappa"] = np.float16(0.5).view(np.uint16)
    else:
        pays["kappa"] = 0.5

    def batch(k):
        paint = pick[k * (n_paint + n_refine):][:n_paint]
        refine = pick[k * (n_paint + n_refine) + n_paint:][:n_refine]
        co = coarse[k * n_coarsen:][:n_coarsen]
        ed = np.zeros(len(paint) + len(refine) + len(co), EDIT_DTYPE)
        a, b = len(paint), len(paint) + len(refine)
        ed["op"][:a], ed["op"][a:b], ed["op"][b:] = 0, 1, 2
        ed["node"] = np.concatenate([paint, refine, co]).astype(np.uint32)
        ed["first_payload"][:a] = np.arange(a)
        ed["first_payload"][a:b] = n_paint + 8 * np.arange(b - a)
        ed["first_payload"][b:] = n_paint + 8 * n_refine + np.arange(len(ed) - b)
        return ed

    batches = [batch(0), batch(1)]
    first = np.zeros(1, EDIT_DTYPE)
    first["node"] = pick[-1]
    torch.cuda.synchronize()
    log(f"pool edits: 2 x {len(batches[0])} edits drawn")
    t = time.perf_counter()
    sess.upload(9, cv)
    torch.cuda.synchronize()
    upload_ms = (time.perf_counter() - t) * 1e3
    log(f"pool edits: upload of the copy {upload_ms:.1f} ms")
    t = time.perf_counter()
    sess.edit(9, first, pays)                             # builds the host mirror
    first_ms = (time.perf_counter() - t) * 1e3
    log(f"pool edits: first edit (mirror build) {first_ms:.1f} ms")
    ms = []
    for ed in batches:
        t = time.perf_counter()
        sess.edit(9, ed, pays)
        ms.append((time.perf_counter() - t) * 1e3)
        log(f"pool edits: batch of {len(ed)} edits {ms[-1]:.1f} ms")
    sess.free(9)
    return dict(paint=int(n_paint), refine=int(n_refine), coarsen=int(n_coarsen),
                edit_ms_growing=round(ms[0], 2), edit_ms=round(ms[1], 2),
                first_edit_ms=round(first_ms, 2), upload_ms=round(upload_ms, 2),
                nodes=int(cv.n_nodes))


def cvx_nodes(sess, canvas_id):
    from paper_1704_02724_amd import cvx
    return cvx.cvx_pool_nodes(sess.ctx, canvas_id)


def stroke_bench(sess, cv, seed):
    """Times brush strokes with deferred refinement (cvx_stroke_begin, then one
    cvx_stroke_step per frame until nothing waits) on a copy of the canvas:
    seeded strokes of a fine, a middle and a large brush radius, and one large
    coarsening stroke (its merges follow its splits)."""
    from canvasgen.strokes import gen_strokes
    torch = sess.torch
    sess.upload(9, cv)
    torch.cuda.synchronize()
    out = []
    for j, (lg, coarsen) in enumerate(((-16, False), (-10, False), (-5, False), (-6, True))):
        st = gen_strokes(np.random.Generator(np.random.PCG64(seed + j)), 1, lg, lg)
        t = time.perf_counter()
        p = sess.stroke_begin(9, st.stamps_of(0), st.rgb[0], st.sigma[0], st.radius[0], 4.0,
                              coarsen=coarsen)
        frames = [round((time.perf_counter() - t) * 1e3, 2)]
        waiting = [p]
        while p:
            t = time.perf_counter()
            p = sess.stroke_step(9)
            frames.append(round((time.perf_counter() - t) * 1e3, 2))
            waiting.append(p)
        row = dict(radius_log2=lg, coarsen=coarsen, stamps=int(len(st.stamps_of(0))),
                   frame_ms=frames, waiting=waiting, nodes=cvx_nodes(sess, 9))
        log(f"stroke: {row}")
        out.append(row)
    sess.free(9)
    return out


def merged_pieces(gpu, n, pieces):
    """Whole-ray leaf sequences from a chord-piece trace (rows (ray, piece),
    ray-major): the pieces concatenated, a leaf cut by a piece boundary
    counted once."""
    ids = gpu["leaf_ids"].reshape(n, pieces, -1)
    cnt = gpu["n_leaves"].reshape(n, pieces).astype(np.int64)
    out_ids = np.zeros((n, ML), np.uint32)
    out_n = np.zeros(n, np.uint32)
    for r in range(n):
        seq = []
        for j in range(pieces):
            part = ids[r, j, :min(int(cnt[r, j]), ML)].tolist()
            if seq and part and part[0] == seq[-1]:
                part = part[1:]
            seq.extend(part)
        out_n[r] = len(seq)
        seq = seq[:ML]
        out_ids[r, :len(seq)] = seq
    return dict(leaf_ids=out_ids, n_leaves=out_n)


def parity_check(sess, w, ids, img, variant, tuning):
    """Leaf sequences and RGBA of `variant` against the oracle on the sampled
    rays, and the naive canvas-global FP32 caster on the same rays.  With
    chord pieces the timed kernel's sequences are the merged piece traces."""
    from oracle import oracle
    views = w.views
    orc = oracle.render(w.canvases, views, ids, max_leaves=ML)
    skip = (orc["flags"] & (oracle.FLAG_NEAR_FACE | oracle.FLAG_TERM_AMBIG)) != 0
    m = np.minimum(orc["n_leaves"], ML).astype(np.int64)
    pos = np.arange(ML)[None, :] < m[:, None]

    def seq_ok(gpu):
        return (gpu["n_leaves"] == orc["n_leaves"]) & np.all(
            (gpu["leaf_ids"] == orc["leaf_ids"]) | ~pos, axis=1)

    gpu = sess.trace(views, ids, ML, variant)
    vi = (ids >> np.uint64(32)).astype(np.int64)
    px = (ids & np.uint64(0xFFFFFFFF)).astype(np.int64)
    offs = np.array([v["out_offset_px"] for v in views], np.int64)
    pix = img[offs[vi] + px]
    rgba_err = np.abs(pix.astype(np.float64) - orc["rgba"]).max(axis=1)
    n = len(ids)
    P = int(tuning.get("chord_pieces", 1))
    if P > 1:
        # the timed kernel splits chords: its sequences are the merged piece
        # traces; the whole-chord kernel is tied to its trace separately
        ok = seq_ok(merged_pieces(sess.trace(views, ids, ML, variant, chord_pieces=P), n, P))
        whole = sess.render(views, variant, use_graph=True,
                            **dict(tuning, chord_pieces=1)).cpu().numpy()
        wpix = whole[offs[vi] + px]
        split_diff = float(np.abs(pix.astype(np.float64) - wpix).max())
    else:
        ok = seq_ok(gpu)
        wpix, split_diff = pix, 0.0
    par = dict(rays=int(n), flagged=int(skip.sum()),
               bit_exact_share=round(float((~skip).mean()), 4),
               seq_mismatch=int((~ok & ~skip).sum()),
               seq_mismatch_flagged=int((~ok & skip).sum()),
               seq_mismatch_whole_chord=int((~seq_ok(gpu) & ~skip).sum()),
               max_rgba_err=float(rgba_err[~skip].max()),
               max_rgba_err_flagged=float(rgba_err[skip].max()) if skip.any() else 0.0,
               trace_equals_render=bool(np.array_equal(gpu["rgba"], wpix)),
               chord_pieces=P, split_vs_whole_max_diff=split_diff,
               gpu_fp64_exit_rays=int(((gpu["flags"] & 2) != 0).sum()),
               mean_leaves=round(float(orc["n_leaves"].mean()), 1))
    par["pass"] = (par["seq_mismatch"] == 0 and par["seq_mismatch_whole_chord"] == 0
                   and par["max_rgba_err"] <= 1e-3 and par["trace_equals_render"]
                   and split_diff <= 1e-3)
    naive = sess.trace(views, ids, ML, "fp32_naive")
    nok = seq_ok(naive)
    nerr = np.abs(naive["rgba"].astype(np.float64) - orc["rgba"]).max(axis=1)
    nv = {"seq_mismatch": int((~nok & ~skip).sum()),
          "seq_mismatch_rate": round(float((~nok & ~skip).sum() / max(1, (~skip).sum())), 4),
          "max_rgba_err": float(nerr[~skip].max()),
          "rays_over_1e-3": int((nerr[~skip] > 1e-3).sum())}
    return par, nv, float(orc["alg_bytes"].mean())


def run_workload(sess, name, args, headline, copy_bps):
    """Every measurement of one workload; the pools are freed at the end."""
    torch = sess.torch
    steps = args.steps if headline else args.extra_steps
    warmup = args.warmup if headline else 2
    t = time.perf_counter()
    w = build_workload(name, args.threads)
    cv = w.canvases
    log(f"[{name}] built: {[c.n_nodes for c in cv]} nodes in {time.perf_counter() - t:.1f}s")
    views = w.views
    rays = w.n_rays
    t = time.perf_counter()
    for i, c in enumerate(cv):
        sess.upload(i, c)
    log(f"[{name}] uploaded in {time.perf_counter() - t:.1f}s")

    tw, th = (int(x) for x in args.tile.split("x"))
    tuning = dict(tile=(tw, th), workgroups=args.workgroups, wg_size=args.wg_size,
                  top_lookup=args.top_lookup, single_queue=args.single_queue)
    tuning64 = dict(tuning)
    if not args.no_autotune:
        t = time.perf_counter()
        reps = args.tune_reps if headline else 1
        tuning, tune_rows = sess.autotune(views, args.variant, reps=reps)
        log(f"[{name}] autotune {args.variant}: {tuning} in {time.perf_counter() - t:.1f}s; "
            "fastest: " + ", ".join(f"{r[0]}x{r[1]}/wg{r[2]}/{r[3]}/top{r[5]}/q{r[6]}/"
                                    f"rpw{r[7]}/min{r[8]}/pieces{r[9]}: {r[4]:.3f}ms"
                                    for r in sorted(tune_rows, key=lambda r: r[4])[:4]))
        plain = [r for r in tune_rows if r[7] == 64 and r[9] == 1]
        extra = [r for r in tune_rows if r[7] > 64 or r[9] > 1]
        if extra:
            log(f"[{name}] on the fastest plain shape ({min(r[4] for r in plain):.3f}ms): "
                + ", ".join(f"rpw{r[7]}/min{r[8]}/pieces{r[9]}: {r[4]:.3f}ms" for r in extra))
        if args.fp64_steps > 0:
            tuning64, _ = sess.autotune(views, "fp64_plain", reps=1)
            log(f"[{name}] autotune fp64_plain: {tuning64}")

    # --- timed: production variant
    out, wall, per = time_variant(sess, views, args.variant, steps, warmup, tuning)
    ms_step = wall * 1e3 / steps
    value = rays / (ms_step * 1e-3) / 1e6
    log(f"[{name}] {args.variant}: {ms_step:.3f} ms/step (events mean {per.mean():.3f}), "
        f"{value:.1f} Mrays/s")

    # --- algorithmic bytes of one launch, counted by the kernel (untimed)
    st = sess.new_stats()
    sess.render(views, args.variant, stats=st, **tuning)
    torch.cuda.synchronize()
    s = st.cpu().numpy().astype(np.float64)
    alg_bytes = 16.0 * s[0] + 8.0 * s[1] + 4.0 * (s[2] + s[3])
    cast_ms = time_cast_kernel(sess, views, args.variant, steps, tuning)
    kernel_s = cast_ms.mean() * 1e-3
    log(f"[{name}] cast kernel alone: mean {cast_ms.mean():.4f} ms, min {cast_ms.min():.4f}, "
        f"max {cast_ms.max():.4f} (the whole render: {per.mean():.4f} ms)")

    # --- FP64 plain baseline on the same GPU
    fp64 = None
    if args.fp64_steps > 0:
        _, wall64, _ = time_variant(sess, views, "fp64_plain", args.fp64_steps, 1, tuning64)
        fp64 = rays / (wall64 / args.fp64_steps) / 1e6
        log(f"[{name}] fp64_plain: {wall64 * 1e3 / args.fp64_steps:.3f} ms/step, "
            f"{fp64:.1f} Mrays/s")

    # --- one launch per view, for the batching comparison
    per_view = None
    pv_steps = args.per_view_steps if args.per_view_steps >= 0 else (3 if len(views) > 2 else 0)
    if pv_steps > 0:
        pv_s, pv_out = time_per_view(sess, views, args.variant, pv_steps, tuning)
        same = bool(torch.equal(pv_out, out))
        per_view = dict(mrays=round(rays / pv_s / 1e6, 2), ms_per_step=round(pv_s * 1e3, 3),
                        launches_per_step=len(views), steps=pv_steps,
                        batched_speedup=round(pv_s / (ms_step * 1e-3), 3), same_image=same)
        log(f"[{name}] per-view launches: {per_view}")
        del pv_out

    # --- parity on a seeded sample (sequences + RGBA) against the oracle, and
    # the naive global-FP32 caster on the same rays
    ids = sample_ids(views, args.parity_sample if headline else args.extra_parity_sample,
                     12345)
    img = out.cpu().numpy()
    parity, naive, mean_b_oracle = parity_check(sess, w, ids, img, args.variant, tuning)
    log(f"[{name}] parity: {parity}")
    log(f"[{name}] naive fp32: {naive}")

    res = dict(workload=name, views=len(views), rays_per_step=int(rays),
               nodes=int(sum(c.n_nodes for c in cv)),
               value=round(value, 2) if parity["pass"] else None,
               value_unchecked=round(value, 2), ms_per_step=round(ms_step, 4), steps=steps,
               tuning=dict(tile="%dx%d" % tuple(tuning["tile"]),
                           workgroups=int(tuning["workgroups"]), wg_size=int(tuning["wg_size"]),
                           top_lookup=int(tuning.get("top_lookup", 0)),
                           single_queue=int(tuning.get("single_queue", 0)),
                           rays_per_wave=int(tuning.get("rays_per_wave", 64)),
                           refill_min=int(tuning.get("refill_min", 0)),
                           chord_pieces=int(tuning.get("chord_pieces", 1)),
                           autotuned=not args.no_autotune),
               fp64_plain_mrays=round(fp64, 2) if fp64 else None,
               speedup_vs_fp64_plain=round(value / fp64, 3) if fp64 else None,
               per_view_launches=per_view, parity=parity, naive_fp32=naive,
               alg_bytes_per_ray=alg_bytes / max(s[0], 1.0),
               alg_bytes_per_ray_oracle_sample=mean_b_oracle,
               alg_bytes_frac=round(alg_bytes / kernel_s / HBM_PEAK, 4),
               kernel_ms=round(kernel_s * 1e3, 4), render_event_ms=round(per.mean(), 4),
               kernel_stats=dict({k: int(v) for k, v in zip(
                   ["rays", "leaves", "outer", "descent", "fp64_exit", "rebase", "steps",
                    "slots"], s[:8])},
                   lane_occupancy=round(float(s[6] / s[7]), 4) if s[7] else None))
    traffic_b, valu_instr = profiled_counts(args.variant, name)
    res["roofline"] = roofline(alg_bytes, kernel_s, traffic_b, valu_instr, copy_bps)

    if name == "depth24" and args.edit_bench:
        res["pool_edit"] = edit_bench(sess, cv[0], 20000, 2000, 500, 99)
        log(f"[{name}] pool edits: {res['pool_edit']}")
        res["pool_edit"]["strokes"] = stroke_bench(sess, cv[0], 123)

    # --- CPU oracle baseline (headline only): a bounded seeded sample
    if headline and not args.no_cpu:
        from oracle import oracle
        n_all = sum(v["W"] * v["H"] for v in views)
        cids = None if n_all <= args.cpu_sample else sample_ids(views, args.cpu_sample, 777)
        n_cpu = n_all if cids is None else len(cids)
        threads = min(16, os.cpu_count() or 1)
        t = time.perf_counter()
        oracle.render(cv, views, cids, threads=threads)
        dt = time.perf_counter() - t
        what = (f"every ray of the workload ({n_all})" if cids is None else
                f"{n_cpu} seeded uniform rays of the same views")
        res["cpu_baseline"] = dict(value=round(n_cpu / dt / 1e6, 4), unit="Mrays/s",
                                   cores=threads, kind="oracle", sample=f"{what}, {dt:.1f}s wall")
        log(f"[{name}] cpu oracle: {res['cpu_baseline']}")

    for i in range(len(cv)):
        sess.free(i)
    del out, img, w, cv
    gc.collect()
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=WORKLOADS)
    ap.add_argument("--extra", default="depth24,depth30,batch,depth24_k10,depth30_k10",
                    help="workloads measured after the headline one, reported under 'configs' "
                         "(comma-separated; empty for none)")
    ap.add_argument("--extra-steps", type=int, default=10)
    ap.add_argument("--extra-parity-sample", type=int, default=32768)
    ap.add_argument("--variant", default="fp32_rebased")
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--parity-sample", type=int, default=65536)
    ap.add_argument("--cpu-sample", type=int, default=1 << 23,
                    help="CPU oracle leg: every ray when the workload has at most this many, "
                         "else this many seeded draws (duplicates removed)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tile", default="8x8")
    ap.add_argument("--workgroups", type=int, default=0)
    ap.add_argument("--wg-size", type=int, default=0)
    ap.add_argument("--top-lookup", type=int, default=0, help="with --no-autotune")
    ap.add_argument("--single-queue", type=int, default=0, help="with --no-autotune")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="use --tile/--workgroups/--wg-size instead of cvx_autotune's pick")
    ap.add_argument("--tune-reps", type=int, default=3)
    ap.add_argument("--edit-bench", type=int, default=1,
                    help="time pool edits and brush strokes on the depth-24 canvas when it is "
                         "measured (0 skips them)")
    ap.add_argument("--per-view-steps", type=int, default=-1,
                    help="steps of the one-launch-per-view comparison (default 3 when the "
                         "workload has more than two views; 0 skips it)")
    ap.add_argument("--issue-probe", action="store_true",
                    help="only run the vector-issue probe (lib/probe_valu: wave64 VALU "
                         "instructions per SIMD per clock for the loop's instruction kinds) "
                         "and print its JSON")
    ap.add_argument("--copy-probe-mb", type=int, default=1024,
                    help="size of the device-to-device copy timed as the measured HBM peak "
                         "(also the reference for hardware byte counters); 0 skips it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the ray caster renders "
              "on one GPU; rays are independent, so more GPUs would split the tiles of a "
              "replicated pool", file=sys.stderr)
        sys.exit(2)
    if args.issue_probe:
        import subprocess
        from paper_1704_02724_amd.build import PROBE_PATH
        r = subprocess.run([PROBE_PATH], capture_output=True, text=True, timeout=120)
        sys.stderr.write(r.stderr)
        print(r.stdout.strip(), flush=True)
        sys.exit(r.returncode)
    extras = [x for x in args.extra.split(",") if x]
    for x in extras:
        if x not in WORKLOADS:
            raise SystemExit(f"unknown workload {x}")

    import torch
    from paper_1704_02724_amd.session import Session

    sess = Session(0)
    copy_bps = None
    if args.copy_probe_mb:
        # measured HBM peak: a device-to-device copy (reads + writes), best of 5
        nb = args.copy_probe_mb << 20
        src = torch.ones(nb, dtype=torch.uint8, device=sess.device)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        best = None
        for _ in range(5):
            s0, e0 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s0.record()
            dst.copy_(src)
            e0.record()
            torch.cuda.synchronize()
            ms = s0.elapsed_time(e0)
            best = ms if best is None else min(best, ms)
        copy_bps = 2.0 * nb / (best * 1e-3)
        log(f"copy probe: {nb} bytes read + {nb} bytes written, best {best:.3f} ms, "
            f"{copy_bps / 1e9:.1f} GB/s")
        del src, dst
        torch.cuda.empty_cache()

    head = run_workload(sess, args.workload, args, True, copy_bps)
    configs = {}
    for x in extras:
        r = run_workload(sess, x, args, False, copy_bps)
        configs[x] = {k: r[k] for k in (
            "value", "value_unchecked", "ms_per_step", "rays_per_step", "views", "nodes",
            "fp64_plain_mrays", "speedup_vs_fp64_plain", "alg_bytes_frac", "parity",
            "naive_fp32", "per_view_launches", "tuning", "kernel_stats")}
        configs[x]["roofline"] = {k: r["roofline"][k] for k in (
            "bound", "frac", "alg_bytes_frac", "hbm_measured_frac", "valu_per_simd_cycle")}
        if "pool_edit" in r:
            configs[x]["pool_edit"] = r["pool_edit"]
    sess.close()

    res = {
        "metric": "Mrays/s at ≤1e-3 RGBA err vs FP64 oracle "
                  "(FP32-rebased batched vs FP64 plain)",
        "value": head["value"],
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict({"workload": args.workload, "views": head["views"],
                        "rays_per_step": head["rays_per_step"], "nodes": head["nodes"],
                        "variant": args.variant, "graph": True}, **head["tuning"]),
        "roofline": head["roofline"],
        "value_unchecked": head["value_unchecked"],
        "fp64_plain_mrays": head["fp64_plain_mrays"],
        "speedup_vs_fp64_plain": head["speedup_vs_fp64_plain"],
        "per_view_launches": head["per_view_launches"],
        "parity": head["parity"],
        "naive_fp32": head["naive_fp32"],
        "alg_bytes_per_ray": head["alg_bytes_per_ray"],
        "alg_bytes_per_ray_oracle_sample": head["alg_bytes_per_ray_oracle_sample"],
        "kernel_stats": head["kernel_stats"],
        "cpu_baseline": head.get("cpu_baseline"),
        "configs": configs,
    }
    print(json.dumps(res), flush=True)


def reap_children():
    """Ends the run with no process of its own left behind: lists any child
    process still alive (the compilers the oracle and the canvas builder may
    start have exited by then, so normally none), then terminates and waits
    for each."""
    try:
        import psutil
    except ImportError:
        return
    kids = psutil.Process().children(recursive=True)
    if not kids:
        return
    def name(k):
        try:
            return f"{k.pid} {' '.join(k.cmdline()[:4])} ({k.status()})"
        except psutil.Error:
            return f"{k.pid} (gone)"
    log("child processes left at exit: " + ", ".join(name(k) for k in kids))
    for k in kids:
        try:
            k.terminate()
        except psutil.NoSuchProcess:
            pass
    _, alive = psutil.wait_procs(kids, timeout=5)
    for k in alive:
        k.kill()
    psutil.wait_procs(alive, timeout=5)


if __name__ == "__main__":
    try:
        main()
    finally:
        reap_children()

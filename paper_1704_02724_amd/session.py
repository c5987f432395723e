"""Convenience wrapper over the C-ABI: torch supplies device memory and the stream.

Marshalling only: uploads hand host arrays to ``cvx_upload_pool``; renders
allocate the output (or trace buffers) as torch tensors on the current device
and call ``cvx_render`` on torch's current stream.
"""
from __future__ import annotations

import numpy as np

from . import cvx


class Session:
    def __init__(self, device: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: libcvx needs a HIP device")
        self.torch = torch
        torch.cuda.set_device(device)
        self.device = torch.device("cuda", device)
        # a stream of our own (default priority): graph capture needs a
        # non-null stream; it is ordered against torch's current stream
        self.stream = torch.cuda.Stream(self.device)
        self.ctx = cvx.cvx_create(device, self.stream.cuda_stream)
        self.descs = {}

    def close(self):
        if self.ctx:
            cvx.cvx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- pools ------------------------------------------------------------
    def upload(self, canvas_id, canvas):
        d = cvx.make_desc(canvas.origin, canvas.root_edge, canvas.R, canvas.max_depth,
                          canvas.leaf_format)
        cvx.cvx_upload_pool(self.ctx, canvas_id, d, canvas.nodes, canvas.leaves)
        self.descs[canvas_id] = d

    def edit(self, canvas_id, edits, payloads):
        """Apply pool edits (cvx_edit_pool); returns the first child id per edit."""
        self.torch.cuda.current_stream(self.device).synchronize()
        return cvx.cvx_edit_pool(self.ctx, canvas_id, edits, payloads)

    def stroke_begin(self, canvas_id, stamps, rgb, sigma, radius, k_refine, coarsen=False):
        """Paint a brush stroke into the existing leaves (cvx_stroke_begin);
        returns the number of leaves waiting for a split."""
        self.torch.cuda.current_stream(self.device).synchronize()
        return cvx.cvx_stroke_begin(self.ctx, canvas_id, stamps, rgb, sigma, radius, k_refine,
                                    coarsen)

    def stroke_step(self, canvas_id):
        """One deferred refinement level of the stroke (cvx_stroke_step)."""
        self.torch.cuda.current_stream(self.device).synchronize()
        return cvx.cvx_stroke_step(self.ctx, canvas_id)

    def free(self, canvas_id):
        cvx.cvx_free_pool(self.ctx, canvas_id)
        self.descs.pop(canvas_id, None)

    # -- stream ordering ----------------------------------------------------
    def _enter(self):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))

    def _leave(self, *tensors):
        self.torch.cuda.current_stream(self.device).wait_stream(self.stream)
        for t in tensors:
            t.record_stream(self.stream)

    # -- render -----------------------------------------------------------
    def out_pixels(self, views):
        return max(v["out_offset_px"] + v["W"] * v["H"] for v in views)

    def render(self, views, variant="fp32_rebased", out=None, out_f64=False, stats=None,
               noalloc=False, **tuning):
        """cvx_render (or, with noalloc, cvx_render_noalloc) into `out`, a new
        tensor when None."""
        torch = self.torch
        n_px = self.out_pixels(views)
        if out is None:
            out = torch.empty((n_px, 4), dtype=torch.float64 if out_f64 else torch.float32,
                              device=self.device)
        varr = cvx.make_views(views)
        opts = cvx.make_opts(variant, out_f64=out_f64,
                             stats_ptr=stats.data_ptr() if stats is not None else 0, **tuning)
        self._enter()
        (cvx.cvx_render_noalloc if noalloc else cvx.cvx_render)(self.ctx, varr, out.data_ptr(),
                                                                 opts)
        self._leave(out, *([stats] if stats is not None else []))
        return out

    def autotune(self, views, variant="fp32_rebased", out=None, reps=3, use_graph=True):
        """Times every candidate launch shape (cvx_autotune); returns the fastest as
        render keyword arguments, and the table of (tile_w, tile_h, wg_size,
        workgroups, ms, top_lookup, single_queue, rays_per_wave, refill_min,
        chord_pieces) rows."""
        torch = self.torch
        if out is None:
            out = torch.empty((self.out_pixels(views), 4), dtype=torch.float32, device=self.device)
        varr = cvx.make_views(views)
        base = cvx.make_opts(variant, use_graph=use_graph)
        self._enter()
        best, rows = cvx.cvx_autotune(self.ctx, varr, out.data_ptr(), base, reps)
        self._leave(out)
        tuning = dict(tile=(best.tile_w, best.tile_h), workgroups=best.workgroups,
                      wg_size=best.wg_size, top_lookup=best.top_lookup,
                      single_queue=best.single_queue, rays_per_wave=best.rays_per_wave or 64,
                      refill_min=best.refill_min if best.rays_per_wave > 64 else 0,
                      chord_pieces=best.chord_pieces or 1)
        return tuning, rows

    def new_stats(self):
        return self.torch.zeros(cvx.CVX_STAT_COUNT, dtype=self.torch.int64, device=self.device)

    def trace(self, views, ray_ids, max_leaves=256, variant="fp32_rebased", len64=False,
              end_point=False, chord_pieces=1):
        """Visited leaves, lengths, flags and RGBA of the listed rays; with
        chord_pieces > 1 one row per (ray, piece), ray-major, rgba = (the
        piece's colour, its transmittance)."""
        torch = self.torch
        ids = torch.from_numpy(np.ascontiguousarray(ray_ids, dtype=np.uint64).view(np.int64))
        ids = ids.to(self.device)
        n = len(ray_ids) * max(1, int(chord_pieces))
        leaf_ids = torch.zeros((n, max(max_leaves, 1)), dtype=torch.int32, device=self.device)
        llen = torch.zeros((n, max(max_leaves, 1)),
                           dtype=torch.float64 if len64 else torch.float32, device=self.device)
        nl = torch.zeros(n, dtype=torch.int32, device=self.device)
        fl = torch.zeros(n, dtype=torch.int32, device=self.device)
        rgba = torch.zeros((n, 4), dtype=torch.float32, device=self.device)
        end = torch.zeros((n, 3), dtype=torch.float64, device=self.device) if end_point else None
        tr = cvx.cvx_trace()
        tr.n = len(ray_ids)
        tr.ray_ids = ids.data_ptr()
        tr.max_leaves = max_leaves
        tr.leaf_ids = leaf_ids.data_ptr()
        tr.local_len = None if len64 else llen.data_ptr()
        tr.local_len64 = llen.data_ptr() if len64 else None
        tr.n_leaves = nl.data_ptr()
        tr.flags = fl.data_ptr()
        tr.rgba = rgba.data_ptr()
        tr.end_point = end.data_ptr() if end is not None else None
        varr = cvx.make_views(views)
        opts = cvx.make_opts(variant, trace=tr, chord_pieces=chord_pieces)
        self._enter()
        cvx.cvx_render(self.ctx, varr, 0, opts)
        self._leave(ids, leaf_ids, llen, nl, fl, rgba, *([end] if end is not None else []))
        torch.cuda.synchronize(self.device)
        res = dict(leaf_ids=leaf_ids.cpu().numpy().view(np.uint32), local_len=llen.cpu().numpy(),
                   n_leaves=nl.cpu().numpy().view(np.uint32), flags=fl.cpu().numpy().view(np.uint32),
                   rgba=rgba.cpu().numpy())
        if end is not None:
            res["end_point"] = end.cpu().numpy()
        return res

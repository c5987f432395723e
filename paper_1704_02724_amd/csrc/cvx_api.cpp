// C-ABI entry points of libcvx: context, pool upload, render, errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cvx_internal.h"

using cvx::CastArgs;
using cvx::CastHeader;
using cvx::DevCanvas;
using cvx::DView;

struct GraphKey {
  uint32_t variant = ~0u, tw = 0, th = 0, wgs = 0, wg = 0;
  bool trace = false, stats = false, out64 = false;
  const void* out = nullptr;
  const void* stats_ptr = nullptr;
  const void* views = nullptr;
  bool operator==(const GraphKey& o) const {
    return variant == o.variant && tw == o.tw && th == o.th && wgs == o.wgs && wg == o.wg &&
           trace == o.trace && stats == o.stats && out64 == o.out64 && out == o.out &&
           stats_ptr == o.stats_ptr && views == o.views;
  }
};

struct cvx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  std::string err;
  DevCanvas canvases[CVX_MAX_CANVASES];
  DView* d_views = nullptr;
  size_t views_cap = 0;
  CastHeader* d_hdr = nullptr;
  DView* h_views = nullptr;  // pinned staging
  size_t h_cap = 0;
  CastHeader* h_hdr = nullptr;  // pinned staging
  hipEvent_t staged{};
  bool staged_pending = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  GraphKey gkey;
};

namespace {

int fail(cvx_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int hip_fail(cvx_ctx* ctx, hipError_t e, const char* where) {
  return fail(ctx, CVX_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define CVX_HIP(call)                                   \
  do {                                                  \
    hipError_t e_ = (call);                             \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
  } while (0)

void free_canvas(DevCanvas& c) {
  if (c.rec) (void)hipFree(c.rec);
  if (c.pay) (void)hipFree(c.pay);
  if (c.top) (void)hipFree(c.top);
  c = DevCanvas();
}

void drop_graph(cvx_ctx* ctx) {
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->gexec = nullptr;
  ctx->graph = nullptr;
  ctx->gkey = GraphKey();
}

uint32_t leaf_bytes(uint32_t fmt) { return fmt == CVX_LEAF_F64 ? 32u : 8u; }

}  // namespace

extern "C" {

const char* cvx_status_str(int s) {
  switch (s) {
    case CVX_OK: return "CVX_OK";
    case CVX_ERR_INVALID_ARG: return "CVX_ERR_INVALID_ARG";
    case CVX_ERR_BAD_POOL: return "CVX_ERR_BAD_POOL";
    case CVX_ERR_OOM: return "CVX_ERR_OOM";
    case CVX_ERR_HIP: return "CVX_ERR_HIP";
    case CVX_ERR_NOT_FOUND: return "CVX_ERR_NOT_FOUND";
    default: return "CVX_ERR_UNKNOWN";
  }
}

const char* cvx_last_error(cvx_ctx* ctx) {
  if (!ctx) return "null context";
  return ctx->err.c_str();
}

int cvx_validate_pool(const cvx_canvas_desc* desc, const cvx_node* nodes, uint64_t n_nodes,
                      const void* leaves, uint64_t n_leaves, char* msg, size_t msg_len) {
  std::string m;
  int rc;
  try {
    rc = cvx::validate_pool(desc, nodes, n_nodes, leaves, n_leaves, nullptr, m);
  } catch (const std::bad_alloc&) {
    rc = CVX_ERR_OOM;
    m = "host allocation failed during validation";
  }
  if (msg && msg_len) {
    std::strncpy(msg, m.c_str(), msg_len - 1);
    msg[msg_len - 1] = 0;
  }
  return rc;
}

int cvx_validate_views(const cvx_view* views, int n_views, const cvx_canvas_desc* const* canvases,
                       int n_canvases, char* msg, size_t msg_len) {
  std::string m;
  int rc = (n_canvases < 0 || (n_canvases > 0 && !canvases))
               ? (m = "bad canvases array", CVX_ERR_INVALID_ARG)
               : cvx::validate_views(views, n_views, canvases, n_canvases, m);
  if (msg && msg_len) {
    std::strncpy(msg, m.c_str(), msg_len - 1);
    msg[msg_len - 1] = 0;
  }
  return rc;
}

int cvx_create(cvx_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return CVX_ERR_INVALID_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return CVX_ERR_HIP;
  if (hip_device < 0 || hip_device >= n) return CVX_ERR_INVALID_ARG;
  cvx_ctx* ctx = new (std::nothrow) cvx_ctx();
  if (!ctx) return CVX_ERR_OOM;
  ctx->device = hip_device;
  ctx->stream = (hipStream_t)hip_stream;
  hipError_t e = hipSetDevice(hip_device);
  hipDeviceProp_t prop;
  if (e == hipSuccess) e = hipGetDeviceProperties(&prop, hip_device);
  if (e == hipSuccess) ctx->n_cu = prop.multiProcessorCount;
  if (e == hipSuccess) e = hipMalloc((void**)&ctx->d_hdr, sizeof(CastHeader));
  if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_hdr, sizeof(CastHeader), 0);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming);
  if (e != hipSuccess) {
    cvx_destroy(ctx);
    return CVX_ERR_HIP;
  }
  *out = ctx;
  return CVX_OK;
}

void cvx_destroy(cvx_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  drop_graph(ctx);
  for (auto& c : ctx->canvases) free_canvas(c);
  if (ctx->d_views) (void)hipFree(ctx->d_views);
  if (ctx->d_hdr) (void)hipFree(ctx->d_hdr);
  if (ctx->h_views) (void)hipHostFree(ctx->h_views);
  if (ctx->h_hdr) (void)hipHostFree(ctx->h_hdr);
  if (ctx->staged) (void)hipEventDestroy(ctx->staged);
  delete ctx;
}

int cvx_upload_pool(cvx_ctx* ctx, int canvas_id, const cvx_canvas_desc* desc,
                    const cvx_node* nodes, uint64_t n_nodes, const void* leaves,
                    uint64_t n_leaves) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  if (canvas_id < 0 || canvas_id >= CVX_MAX_CANVASES)
    return fail(ctx, CVX_ERR_INVALID_ARG, "canvas_id out of range");
  cvx::PoolPlan plan;
  std::string msg;
  int rc;
  try {
    rc = cvx::validate_pool(desc, nodes, n_nodes, leaves, n_leaves, &plan, msg);
  } catch (const std::bad_alloc&) {
    return fail(ctx, CVX_ERR_OOM, "host allocation failed during validation");
  }
  if (rc) return fail(ctx, rc, msg);
  CVX_HIP(hipSetDevice(ctx->device));

  const uint64_t lb = leaf_bytes(desc->leaf_format);
  const uint32_t top_depth = cvx::top_table_depth(desc->R, plan.depth);
  const uint64_t top_side = (uint64_t)desc->R << top_depth;
  const uint64_t top_bytes = top_depth ? top_side * top_side * top_side * 4 : 0;
  const uint64_t rec_bytes = n_nodes * 16, pay_bytes = n_nodes * lb + top_bytes;
  const uint64_t tmp_bytes = n_nodes * 8 + std::max<uint64_t>(n_leaves, 1) * lb +
                             std::max<uint64_t>(plan.order.size(), 1) * 4;
  size_t free_b = 0, total_b = 0;
  CVX_HIP(hipMemGetInfo(&free_b, &total_b));
  if (rec_bytes + pay_bytes + tmp_bytes + (64ull << 20) > free_b)
    return fail(ctx, CVX_ERR_OOM, "pool needs " + std::to_string(rec_bytes + pay_bytes + tmp_bytes) +
                                      " device bytes, " + std::to_string(free_b) + " free");

  DevCanvas nc;
  nc.desc = *desc;
  nc.n_nodes = n_nodes;
  nc.depth = plan.depth;
  void *raw = nullptr, *rawl = nullptr, *ord = nullptr;
  auto cleanup = [&]() {
    if (raw) (void)hipFree(raw);
    if (rawl) (void)hipFree(rawl);
    if (ord) (void)hipFree(ord);
    free_canvas(nc);
  };
  hipError_t e = hipSuccess;
  const char* where = "";
#define STEP(call)               \
  if (e == hipSuccess) {         \
    e = (call);                  \
    if (e != hipSuccess) where = #call; \
  }
  STEP(hipMalloc(&nc.rec, rec_bytes));
  STEP(hipMalloc(&nc.pay, n_nodes * lb));
  if (top_bytes) STEP(hipMalloc((void**)&nc.top, top_bytes));
  STEP(hipMalloc(&raw, n_nodes * 8));
  STEP(hipMalloc(&rawl, std::max<uint64_t>(n_leaves, 1) * lb));
  STEP(hipMalloc(&ord, std::max<uint64_t>(plan.order.size(), 1) * 4));
  if (e == hipErrorOutOfMemory) {
    cleanup();
    return fail(ctx, CVX_ERR_OOM, "device allocation failed");
  }
  STEP(hipMemsetAsync(nc.rec, 0, rec_bytes, ctx->stream));
  STEP(hipMemsetAsync(nc.pay, 0, n_nodes * lb, ctx->stream));
  STEP(hipMemcpyAsync(raw, nodes, n_nodes * 8, hipMemcpyHostToDevice, ctx->stream));
  if (n_leaves) STEP(hipMemcpyAsync(rawl, leaves, n_leaves * lb, hipMemcpyHostToDevice, ctx->stream));
  STEP(hipMemcpyAsync(ord, plan.order.data(), plan.order.size() * 4, hipMemcpyHostToDevice,
                      ctx->stream));
  for (uint32_t lvl = 0; e == hipSuccess && lvl + 1 < plan.level_off.size(); ++lvl) {
    int le = cvx::launch_relayout_level(ctx->stream, (const uint32_t*)ord, plan.level_off[lvl],
                                        plan.level_off[lvl + 1], lvl, raw, rawl, desc->leaf_format,
                                        nc.rec, nc.pay, desc->R);
    if (le != hipSuccess) {
      e = (hipError_t)le;
      where = "k_relayout_level";
    }
  }
  if (e == hipSuccess && top_bytes) {
    nc.top_depth = top_depth;
    int le = cvx::launch_top_table(ctx->stream, nc.rec, n_nodes, desc->R, top_depth, nc.top);
    if (le != hipSuccess) {
      e = (hipError_t)le;
      where = "k_top_table";
    }
  }
  STEP(hipStreamSynchronize(ctx->stream));
#undef STEP
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(ctx, e, where);
  }
  (void)hipFree(raw);
  (void)hipFree(rawl);
  (void)hipFree(ord);
  raw = rawl = ord = nullptr;
  nc.present = true;
  nc.bytes = rec_bytes + pay_bytes;
  free_canvas(ctx->canvases[canvas_id]);
  ctx->canvases[canvas_id] = nc;
  return CVX_OK;
}

int cvx_free_pool(cvx_ctx* ctx, int canvas_id) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  if (canvas_id < 0 || canvas_id >= CVX_MAX_CANVASES)
    return fail(ctx, CVX_ERR_INVALID_ARG, "canvas_id out of range");
  if (!ctx->canvases[canvas_id].present) return fail(ctx, CVX_ERR_NOT_FOUND, "no pool under canvas_id");
  CVX_HIP(hipSetDevice(ctx->device));
  CVX_HIP(hipStreamSynchronize(ctx->stream));
  free_canvas(ctx->canvases[canvas_id]);
  return CVX_OK;
}

int cvx_pool_bytes(cvx_ctx* ctx, int canvas_id, uint64_t* bytes) {
  if (!ctx || !bytes) return CVX_ERR_INVALID_ARG;
  if (canvas_id < 0 || canvas_id >= CVX_MAX_CANVASES) return fail(ctx, CVX_ERR_INVALID_ARG, "canvas_id out of range");
  if (!ctx->canvases[canvas_id].present) return fail(ctx, CVX_ERR_NOT_FOUND, "no pool under canvas_id");
  *bytes = ctx->canvases[canvas_id].bytes;
  return CVX_OK;
}

int cvx_render(cvx_ctx* ctx, const cvx_view* views, int n_views, void* out_dev,
               const cvx_render_opts* opts) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  cvx_render_opts o{};
  if (opts) o = *opts;
  if (o.variant > CVX_VARIANT_FP32_NAIVE) return fail(ctx, CVX_ERR_INVALID_ARG, "unknown variant");
  uint32_t tw = o.tile_w ? o.tile_w : 8, th = o.tile_h ? o.tile_h : 8;
  if (tw * th != 64 || tw == 0 || th == 0)
    return fail(ctx, CVX_ERR_INVALID_ARG, "tile_w * tile_h must be 64");
  uint32_t wg = o.wg_size ? o.wg_size : 256;
  if (wg != 64 && wg != 128 && wg != 256)
    return fail(ctx, CVX_ERR_INVALID_ARG, "wg_size must be 64, 128 or 256");
  uint32_t wgs = o.workgroups ? o.workgroups : (uint32_t)ctx->n_cu * (2048u / wg);
  if (wgs > (1u << 20)) return fail(ctx, CVX_ERR_INVALID_ARG, "too many workgroups");
  if (o.top_lookup > 1) return fail(ctx, CVX_ERR_INVALID_ARG, "top_lookup must be 0 or 1");
  if (o.single_queue > 1) return fail(ctx, CVX_ERR_INVALID_ARG, "single_queue must be 0 or 1");
  if (o.out_f64 && o.variant != CVX_VARIANT_FP64_PLAIN)
    return fail(ctx, CVX_ERR_INVALID_ARG, "out_f64 needs the FP64_PLAIN variant");
  const cvx_trace* tr = o.trace;
  if (tr) {
    if (!tr->ray_ids || !tr->n_leaves || !tr->flags || !tr->rgba ||
        (tr->max_leaves && !tr->leaf_ids) || tr->n == 0 || tr->n > (1ull << 36))
      return fail(ctx, CVX_ERR_INVALID_ARG, "incomplete trace buffers");
  } else if (!out_dev) {
    return fail(ctx, CVX_ERR_INVALID_ARG, "out_dev is NULL");
  }
  if (o.use_graph && !ctx->stream)
    return fail(ctx, CVX_ERR_INVALID_ARG, "use_graph needs a non-null stream");

  const cvx_canvas_desc* descs[CVX_MAX_CANVASES];
  for (int i = 0; i < CVX_MAX_CANVASES; ++i)
    descs[i] = ctx->canvases[i].present ? &ctx->canvases[i].desc : nullptr;
  std::string msg;
  int rc = cvx::validate_views(views, n_views, descs, CVX_MAX_CANVASES, msg);
  if (rc) return fail(ctx, rc, msg);
  for (int i = 0; i < n_views; ++i) {
    const DevCanvas& c = ctx->canvases[views[i].canvas_id];
    if (o.variant != CVX_VARIANT_FP64_PLAIN && c.desc.leaf_format != CVX_LEAF_RGBA8_F16)
      return fail(ctx, CVX_ERR_INVALID_ARG,
                  "view " + std::to_string(i) + ": FP32 variants read RGBA8_F16 leaves only");
  }

  CVX_HIP(hipSetDevice(ctx->device));
  if (ctx->staged_pending) {
    CVX_HIP(hipEventSynchronize(ctx->staged));
    ctx->staged_pending = false;
  }
  if ((size_t)n_views > ctx->h_cap) {
    if (ctx->h_views) (void)hipHostFree(ctx->h_views);
    ctx->h_views = nullptr;
    ctx->h_cap = 0;
    CVX_HIP(hipHostMalloc((void**)&ctx->h_views, sizeof(DView) * n_views, 0));
    ctx->h_cap = n_views;
  }
  if ((size_t)n_views > ctx->views_cap) {
    CVX_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->d_views) (void)hipFree(ctx->d_views);
    ctx->d_views = nullptr;
    ctx->views_cap = 0;
    size_t cap = std::max<size_t>(64, n_views);
    CVX_HIP(hipMalloc((void**)&ctx->d_views, sizeof(DView) * cap));
    ctx->views_cap = cap;
    drop_graph(ctx);
  }
  uint64_t first = 0;
  for (int i = 0; i < n_views; ++i) {
    const cvx_view& v = views[i];
    const DevCanvas& c = ctx->canvases[v.canvas_id];
    DView& dv = ctx->h_views[i];
    std::memset(&dv, 0, sizeof(dv));
    dv.rec = c.rec;
    dv.pay = c.pay;
    dv.R = c.desc.R;
    dv.fmt = c.desc.leaf_format;
    dv.max_depth = c.depth;
    for (int k = 0; k < 3; ++k) {
      dv.o[k] = (v.eye[k] - c.desc.origin[k]) / c.desc.root_edge;
      dv.right[k] = v.right[k];
      dv.up[k] = v.up[k];
      dv.fwd[k] = v.fwd[k];
    }
    dv.tan_x = v.tan_half_fov_x;
    dv.tan_y = v.tan_half_fov_y;
    dv.W = v.W;
    dv.H = v.H;
    dv.out_off = v.out_offset_px;
    dv.alpha_stop = v.alpha_stop;
    dv.tiles_x = (v.W + tw - 1) / tw;
    uint64_t tiles_y = (v.H + th - 1) / th;
    dv.first_tile = first;
    first += (uint64_t)dv.tiles_x * tiles_y;
    uint64_t cap = 3ull * c.desc.R * (1ull << std::min<uint32_t>(c.depth, 40)) + 16;
    dv.max_steps = (uint32_t)std::min<uint64_t>(cap, 1ull << 22);
    dv.n_nodes = (uint32_t)c.n_nodes;
    const bool top = o.top_lookup == 0 && c.top_depth > 0;
    dv.top_depth = top ? c.top_depth : 0;
    dv.top = top ? c.top : nullptr;
  }
  CastHeader& H = *ctx->h_hdr;
  H.total_work = tr ? (tr->n + 63) / 64 : first;
  H.n_rays = tr ? tr->n : 0;
  H.n_views = (uint32_t)n_views;
  H.n_queues = o.single_queue ? 1u : cvx::CVX_NQ;
  for (auto& q : H.queue) q.next = 0;
  if (H.total_work >= (1ull << 32)) return fail(ctx, CVX_ERR_INVALID_ARG, "too much work in one call");
  CVX_HIP(hipMemcpyAsync(ctx->d_views, ctx->h_views, sizeof(DView) * n_views,
                         hipMemcpyHostToDevice, ctx->stream));
  CVX_HIP(hipMemcpyAsync(ctx->d_hdr, ctx->h_hdr, sizeof(CastHeader), hipMemcpyHostToDevice,
                         ctx->stream));
  CVX_HIP(hipEventRecord(ctx->staged, ctx->stream));
  ctx->staged_pending = true;

  CastArgs a{};
  a.views = ctx->d_views;
  a.hdr = ctx->d_hdr;
  a.out = out_dev;
  a.stats = o.stats;
  a.tile_w = tw;
  a.tile_h = th;
  if (tr) {
    a.ray_ids = tr->ray_ids;
    a.max_leaves = tr->max_leaves;
    a.leaf_ids = tr->leaf_ids;
    a.local_len = tr->local_len;
    a.local_len64 = tr->local_len64;
    a.n_leaves = tr->n_leaves;
    a.flags = tr->flags;
    a.trace_rgba = tr->rgba;
  }
  const bool stats = o.stats != nullptr;
  if (!o.use_graph || tr) {
    int le = cvx::launch_reset(ctx->stream, ctx->d_hdr);
    if (le != hipSuccess) return hip_fail(ctx, (hipError_t)le, "k_reset");
    le = cvx::launch_cast(ctx->stream, o.variant, tr != nullptr, stats, o.out_f64 != 0, a, wgs, wg);
    if (le != hipSuccess) return hip_fail(ctx, (hipError_t)le, "k_cast");
    return CVX_OK;
  }
  GraphKey key;
  key.variant = o.variant;
  key.tw = tw;
  key.th = th;
  key.wgs = wgs;
  key.wg = wg;
  key.trace = false;
  key.stats = stats;
  key.out64 = o.out_f64 != 0;
  key.out = out_dev;
  key.stats_ptr = o.stats;
  key.views = ctx->d_views;
  if (!ctx->gexec || !(key == ctx->gkey)) {
    drop_graph(ctx);
    CVX_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    int le = cvx::launch_reset(ctx->stream, ctx->d_hdr);
    if (le == hipSuccess)
      le = cvx::launch_cast(ctx->stream, o.variant, false, stats, o.out_f64 != 0, a, wgs, wg);
    hipGraph_t g = nullptr;
    hipError_t ee = hipStreamEndCapture(ctx->stream, &g);
    if (le != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(ctx, (hipError_t)le, "graph capture launch");
    }
    if (ee != hipSuccess) return hip_fail(ctx, ee, "hipStreamEndCapture");
    ctx->graph = g;
    CVX_HIP(hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0));
    ctx->gkey = key;
  }
  CVX_HIP(hipGraphLaunch(ctx->gexec, ctx->stream));
  return CVX_OK;
}

int cvx_autotune(cvx_ctx* ctx, const cvx_view* views, int n_views, void* out_dev,
                 const cvx_render_opts* base, uint32_t reps, cvx_render_opts* best,
                 cvx_tune_result* results, uint32_t max_results, uint32_t* n_results) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!best) return fail(ctx, CVX_ERR_INVALID_ARG, "best is NULL");
  if (reps < 1 || reps > 1000) return fail(ctx, CVX_ERR_INVALID_ARG, "reps must be in [1, 1000]");
  if (results == nullptr && max_results != 0)
    return fail(ctx, CVX_ERR_INVALID_ARG, "results is NULL but max_results > 0");
  cvx_render_opts b{};
  if (base) b = *base;
  if (b.trace || b.stats)
    return fail(ctx, CVX_ERR_INVALID_ARG, "autotune times plain renders: no trace, no stats");
  static const uint32_t kTiles[][2] = {{8, 8}, {16, 4}, {4, 16}, {32, 2}};
  static const uint32_t kWg[] = {64, 128, 256};
  static const uint32_t kWavesPerCu[] = {16, 28, 32, 64};
  static const uint32_t kTop[] = {0, 1};
  static const uint32_t kQueue[] = {0, 1};
  CVX_HIP(hipSetDevice(ctx->device));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CVX_HIP(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(ctx, he, "hipEventCreate");
  }
  int rc = CVX_OK;
  float best_ms = 0.0f;
  bool have = false;
  uint32_t count = 0;
  for (uint32_t sq : kQueue) {
  for (uint32_t top : kTop) {
  for (const auto& t : kTiles) {
    for (uint32_t wg : kWg) {
      for (uint32_t wpc : kWavesPerCu) {
        if (rc != CVX_OK) break;
        cvx_render_opts o = b;
        o.tile_w = t[0];
        o.tile_h = t[1];
        o.wg_size = wg;
        o.workgroups = (uint32_t)ctx->n_cu * wpc * 64u / wg;
        o.top_lookup = top;
        o.single_queue = sq;
        rc = cvx_render(ctx, views, n_views, out_dev, &o);  // warm-up, captures the graph
        if (rc != CVX_OK) break;
        if ((he = hipEventRecord(e0, ctx->stream)) != hipSuccess) {
          rc = hip_fail(ctx, he, "hipEventRecord");
          break;
        }
        for (uint32_t r = 0; r < reps && rc == CVX_OK; ++r)
          rc = cvx_render(ctx, views, n_views, out_dev, &o);
        if (rc != CVX_OK) break;
        float ms = 0.0f;
        if ((he = hipEventRecord(e1, ctx->stream)) != hipSuccess ||
            (he = hipEventSynchronize(e1)) != hipSuccess ||
            (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) {
          rc = hip_fail(ctx, he, "timing a candidate");
          break;
        }
        ms /= (float)reps;
        if (count < max_results) {
          cvx_tune_result& x = results[count];
          x.tile_w = o.tile_w;
          x.tile_h = o.tile_h;
          x.wg_size = o.wg_size;
          x.workgroups = o.workgroups;
          x.ms = ms;
          x.top_lookup = o.top_lookup;
          x.single_queue = o.single_queue;
        }
        ++count;
        if (!have || ms < best_ms) {
          have = true;
          best_ms = ms;
          *best = o;
        }
      }
    }
  }
  }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (n_results) *n_results = count;
  return rc;
}

}  // extern "C"

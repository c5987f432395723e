// C-ABI entry points of libcvx: context, pool upload, render and launch
// autotuning, pool edits and brush strokes, diagnostics, errors.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "cvx_internal.h"

using cvx::CastArgs;
using cvx::CastHeader;
using cvx::DevCanvas;
using cvx::DView;

struct GraphKey {
  uint32_t variant = ~0u, tw = 0, th = 0, wgs = 0, wg = 0, item_tiles = 1, refill_min = 0,
           pieces = 1;
  bool trace = false, stats = false, out64 = false, small = false, per_ray_start = false;
  const void* out = nullptr;
  const void* stats_ptr = nullptr;
  const void* views = nullptr;
  const void* split_tmp = nullptr;
  bool operator==(const GraphKey& o) const {
    return variant == o.variant && tw == o.tw && th == o.th && wgs == o.wgs && wg == o.wg &&
           item_tiles == o.item_tiles && refill_min == o.refill_min && pieces == o.pieces &&
           split_tmp == o.split_tmp &&
           trace == o.trace && stats == o.stats && out64 == o.out64 && small == o.small &&
           per_ray_start == o.per_ray_start &&
           out == o.out && stats_ptr == o.stats_ptr && views == o.views;
  }
};

struct cvx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  std::string err;
  DevCanvas canvases[CVX_MAX_CANVASES];
  // a render call's header and view table, staged in one pinned host block
  // and copied by one transfer into one device block: CastHeader, then
  // stage_cap view records
  void* d_stage = nullptr;
  void* h_stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t staged{};
  bool staged_pending = false;
  // chord pieces of split renders: (colour, T) per pixel and piece
  void* d_split = nullptr;
  size_t split_cap = 0;
  // cvx_render_noalloc: the library's device scratch array on this device
  // (a CastHeader, then the view table) and a pinned host copy of it
  void* d_scratch = nullptr;
  void* h_scratch = nullptr;
  hipEvent_t scratch_staged{};
  bool scratch_pending = false;
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
  if (c.mark) (void)hipFree(c.mark);
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
  const size_t stage0 = sizeof(CastHeader) + 64 * sizeof(DView);
  if (e == hipSuccess) e = hipMalloc(&ctx->d_stage, stage0);
  if (e == hipSuccess) e = hipHostMalloc(&ctx->h_stage, stage0, 0);
  if (e == hipSuccess) ctx->stage_cap = 64;
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->staged, hipEventDisableTiming);
  // the allocation-free render path: the address of this device's scratch
  // array (looked up once per device, with the device current) and the
  // pinned host copy its calls stage through
  if (e == hipSuccess) e = (hipError_t)cvx::scratch_address(hip_device, &ctx->d_scratch);
  if (e == hipSuccess) e = hipHostMalloc(&ctx->h_scratch, cvx::CVX_SCRATCH_BYTES, 0);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->scratch_staged, hipEventDisableTiming);
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
  if (ctx->d_stage) (void)hipFree(ctx->d_stage);
  if (ctx->d_split) (void)hipFree(ctx->d_split);
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  if (ctx->staged) (void)hipEventDestroy(ctx->staged);
  if (ctx->h_scratch) (void)hipHostFree(ctx->h_scratch);
  if (ctx->scratch_staged) (void)hipEventDestroy(ctx->scratch_staged);
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
  // nodes outside the tree keep x = CVX_FREE and null links
  STEP(hipMemsetAsync(nc.rec, 0xff, rec_bytes, ctx->stream));
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
  nc.cap_nodes = n_nodes;
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

}  // extern "C"

namespace {

// Launch shape and mode of one render call, from its options.
struct RenderPlan {
  uint32_t tw = 8, th = 8, wg = 256, wgs = 0;
  uint32_t item_tiles = 1, refill_min = 32;  // lane refill of the FP32 render (item_tiles > 1)
  uint32_t pieces = 1;  // chord pieces per ray of the FP32 render or trace (views that run to
                        // the canvas exit; 1: unsplit)
};

// Checks the options and views of a render call (nothing is launched on an
// error).
int render_check(cvx_ctx* ctx, const cvx_view* views, int n_views, const void* out_dev,
                 const cvx_render_opts& o, RenderPlan& p) {
  if (o.variant > CVX_VARIANT_FP16_CELL_LOCAL)
    return fail(ctx, CVX_ERR_INVALID_ARG, "unknown variant");
  p.tw = o.tile_w ? o.tile_w : 8;
  p.th = o.tile_h ? o.tile_h : 8;
  if (p.tw * p.th != 64 || p.tw == 0 || p.th == 0)
    return fail(ctx, CVX_ERR_INVALID_ARG, "tile_w * tile_h must be 64");
  p.wg = o.wg_size ? o.wg_size : 256;
  if (p.wg != 64 && p.wg != 128 && p.wg != 256)
    return fail(ctx, CVX_ERR_INVALID_ARG, "wg_size must be 64, 128 or 256");
  p.wgs = o.workgroups ? o.workgroups : (uint32_t)ctx->n_cu * (2048u / p.wg);
  if (p.wgs > (1u << 20)) return fail(ctx, CVX_ERR_INVALID_ARG, "too many workgroups");
  if (o.top_lookup > 1) return fail(ctx, CVX_ERR_INVALID_ARG, "top_lookup must be 0 or 1");
  if (o.single_queue > 1) return fail(ctx, CVX_ERR_INVALID_ARG, "single_queue must be 0 or 1");
  if (o.per_ray_start > 1) return fail(ctx, CVX_ERR_INVALID_ARG, "per_ray_start must be 0 or 1");
  if (o.wide_offsets > 1) return fail(ctx, CVX_ERR_INVALID_ARG, "wide_offsets must be 0 or 1");
  const uint32_t rpw = o.rays_per_wave ? o.rays_per_wave : 64u;
  if (rpw % 64u != 0 || rpw > 1024u)
    return fail(ctx, CVX_ERR_INVALID_ARG, "rays_per_wave must be a multiple of 64 up to 1024");
  if (o.refill_min > 64) return fail(ctx, CVX_ERR_INVALID_ARG, "refill_min must be in 0..64");
  // trace and stats renders run one ray per lane (the same per-ray results)
  const bool refill = o.variant == CVX_VARIANT_FP32_REBASED && !o.trace && !o.stats && rpw > 64u;
  p.item_tiles = refill ? rpw / 64u : 1u;
  p.refill_min = refill ? (o.refill_min ? o.refill_min : 32u) : 0u;
  const uint32_t pieces = o.chord_pieces ? o.chord_pieces : 1u;
  if (pieces != 1 && pieces != 2 && pieces != 4 && pieces != 8)
    return fail(ctx, CVX_ERR_INVALID_ARG, "chord_pieces must be 1, 2, 4 or 8");
  if (pieces > 1 && o.variant != CVX_VARIANT_FP32_REBASED)
    return fail(ctx, CVX_ERR_INVALID_ARG, "chord_pieces needs the FP32_REBASED variant");
  if (pieces > 1 && rpw > 64u)
    return fail(ctx, CVX_ERR_INVALID_ARG, "chord_pieces and rays_per_wave > 64 do not combine");
  if (pieces > 1 && o.stats && o.trace)
    return fail(ctx, CVX_ERR_INVALID_ARG, "chord_pieces with trace takes no stats");
  // stats renders count the unsplit traversal (the same per-ray counts)
  p.pieces = o.stats ? 1u : pieces;
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
  if (o.cast_events && o.use_graph)
    return fail(ctx, CVX_ERR_INVALID_ARG, "cast_events are recorded by eager launches only");

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
  return CVX_OK;
}

// Where a render call stages its header and view table: a pinned host block
// and its device destination, each a CastHeader followed by the views, so
// that one copy moves both.
struct RenderStage {
  DView* h_views;
  CastHeader* h_hdr;
  DView* d_views;
  CastHeader* d_hdr;
  hipEvent_t staged;  // recorded after the copy; the host staging is reused only after it
  bool* staged_pending;
  bool split_ok;           // a split render may use the context's piece buffer
  const char* split_why;   // the error otherwise
};

// Fills the staged views and header, copies them to the device and launches
// the view-start, queue-reset and cast kernels, eagerly or through the
// context's graph.
int render_launch(cvx_ctx* ctx, const cvx_view* views, int n_views, void* out_dev,
                  const cvx_render_opts& o, const RenderPlan& p, const RenderStage& st) {
  const cvx_trace* tr = o.trace;
  uint64_t first = 0;
  for (int i = 0; i < n_views; ++i) {
    const cvx_view& v = views[i];
    const DevCanvas& c = ctx->canvases[v.canvas_id];
    DView& dv = st.h_views[i];
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
    dv.two_w = 2.0 / (double)v.W;
    dv.two_h = 2.0 / (double)v.H;
    dv.W = v.W;
    dv.H = v.H;
    dv.out_off = v.out_offset_px;
    dv.alpha_stop = v.alpha_stop;
    dv.t_stop = (float)(1.0 - (double)v.alpha_stop);
    dv.tiles_x = (v.W + p.tw - 1) / p.tw;
    uint64_t tiles_y = (v.H + p.th - 1) / p.th;
    // work items before this view: tiles, or with lane refill groups of
    // item_tiles tiles (an item never straddles views)
    dv.first_tile = first;
    first += ((uint64_t)dv.tiles_x * tiles_y + p.item_tiles - 1) / p.item_tiles;
    // chord pieces only where rays run to the canvas exit (an opacity stop
    // ends a ray part-way, which a later piece cannot know)
    dv.pieces = (p.pieces > 1 && !(v.alpha_stop < 1.0f)) ? p.pieces : 1u;
    if (!tr) first += ((uint64_t)dv.tiles_x * tiles_y) * (dv.pieces - 1u);  // items: tile x piece
    uint64_t cap = 3ull * c.desc.R * (1ull << std::min<uint32_t>(c.depth, 40)) + 16;
    dv.max_steps = (uint32_t)std::min<uint64_t>(cap, 1ull << 22);
    dv.n_nodes = (uint32_t)c.n_nodes;
    const bool top = o.top_lookup == 0 && c.top_depth > 0;
    dv.top_depth = top ? c.top_depth : 0;
    dv.top = top ? c.top : nullptr;
    dv.start_ok = 0;  // set on the device by k_view_starts
  }
  CastHeader& H = *st.h_hdr;
  // trace rows: one per ray, or per (ray, piece) with chord pieces
  const uint64_t rows = tr ? tr->n * p.pieces : 0;
  H.total_work = tr ? (rows + 63) / 64 : first;
  H.n_rays = rows;
  H.n_views = (uint32_t)n_views;
  H.n_queues = o.single_queue ? 1u : cvx::CVX_NQ;
  for (auto& q : H.queue) q.next = 0;
  if (H.total_work >= (1ull << 32)) return fail(ctx, CVX_ERR_INVALID_ARG, "too much work in one call");
  // one transfer; it also zeroes the queue heads for this call
  CVX_HIP(hipMemcpyAsync(st.d_hdr, st.h_hdr, sizeof(CastHeader) + sizeof(DView) * n_views,
                         hipMemcpyHostToDevice, ctx->stream));
  CVX_HIP(hipEventRecord(st.staged, ctx->stream));
  *st.staged_pending = true;

  CastArgs a{};
  a.views = st.d_views;
  a.hdr = st.d_hdr;
  a.out = out_dev;
  a.stats = o.stats;
  a.tile_w = p.tw;
  a.tile_h = p.th;
  a.item_tiles = p.item_tiles;
  a.refill_min = p.refill_min;
  a.pieces = p.pieces;
  a.small_pools = o.wide_offsets ? 0u : 1u;
  for (int i = 0; i < n_views; ++i)
    if (ctx->canvases[views[i].canvas_id].n_nodes > (1ull << 28)) a.small_pools = 0;
  if (tr) {
    a.ray_ids = tr->ray_ids;
    a.max_leaves = tr->max_leaves;
    a.leaf_ids = tr->leaf_ids;
    a.local_len = tr->local_len;
    a.local_len64 = tr->local_len64;
    a.n_leaves = tr->n_leaves;
    a.flags = tr->flags;
    a.trace_rgba = tr->rgba;
    a.end_point = tr->end_point;
  }
  const bool stats = o.stats != nullptr;
  const uint32_t shared_start = o.per_ray_start ? 0u : 1u;
  // a split render writes its pieces to the context's buffer, merged after
  bool merge = false;
  if (!tr && p.pieces > 1) {
    uint64_t px_end = 0;
    for (int i = 0; i < n_views; ++i)
      if (st.h_views[i].pieces > 1)
        px_end = std::max<uint64_t>(px_end, views[i].out_offset_px +
                                                (uint64_t)views[i].W * views[i].H);
    if (px_end) {
      if (!st.split_ok) return fail(ctx, CVX_ERR_INVALID_ARG, st.split_why);
      const size_t need = (size_t)px_end * p.pieces * 16;
      if (need > ctx->split_cap) {
        CVX_HIP(hipStreamSynchronize(ctx->stream));
        if (ctx->d_split) (void)hipFree(ctx->d_split);
        ctx->d_split = nullptr;
        ctx->split_cap = 0;
        CVX_HIP(hipMalloc(&ctx->d_split, need));
        ctx->split_cap = need;
        drop_graph(ctx);
      }
      merge = true;
    }
  }
  a.split_tmp = merge ? ctx->d_split : nullptr;
  if (!o.use_graph || tr) {
    int le = cvx::launch_view_starts(ctx->stream, st.d_views, st.d_hdr, shared_start);
    if (le != hipSuccess) return hip_fail(ctx, (hipError_t)le, "k_view_starts");
    const hipEvent_t* ev = (const hipEvent_t*)o.cast_events;
    if (ev) CVX_HIP(hipEventRecord(ev[0], ctx->stream));
    le = cvx::launch_cast(ctx->stream, o.variant, tr != nullptr, stats, o.out_f64 != 0, a, p.wgs,
                          p.wg);
    if (le != hipSuccess) return hip_fail(ctx, (hipError_t)le, "k_cast");
    if (ev) CVX_HIP(hipEventRecord(ev[1], ctx->stream));
    if (merge) {
      le = cvx::launch_merge_pieces(ctx->stream, st.d_views, st.d_hdr, (uint32_t)n_views,
                                    ctx->d_split, out_dev, p.pieces);
      if (le != hipSuccess) return hip_fail(ctx, (hipError_t)le, "k_merge_pieces");
    }
    return CVX_OK;
  }
  GraphKey key;
  key.variant = o.variant;
  key.tw = p.tw;
  key.th = p.th;
  key.wgs = p.wgs;
  key.wg = p.wg;
  key.item_tiles = p.item_tiles;
  key.refill_min = p.refill_min;
  key.pieces = p.pieces;
  key.split_tmp = a.split_tmp;
  key.trace = false;
  key.stats = stats;
  key.out64 = o.out_f64 != 0;
  key.small = a.small_pools != 0;
  key.per_ray_start = o.per_ray_start != 0;
  key.out = out_dev;
  key.stats_ptr = o.stats;
  key.views = st.d_views;
  if (!ctx->gexec || !(key == ctx->gkey)) {
    drop_graph(ctx);
    CVX_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    int le = cvx::launch_view_starts(ctx->stream, st.d_views, st.d_hdr, shared_start);
    if (le == hipSuccess)
      le = cvx::launch_cast(ctx->stream, o.variant, false, stats, o.out_f64 != 0, a, p.wgs, p.wg);
    if (le == hipSuccess && merge)
      le = cvx::launch_merge_pieces(ctx->stream, st.d_views, st.d_hdr, (uint32_t)n_views,
                                    ctx->d_split, out_dev, p.pieces);
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

}  // namespace

extern "C" {

int cvx_render(cvx_ctx* ctx, const cvx_view* views, int n_views, void* out_dev,
               const cvx_render_opts* opts) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  cvx_render_opts o{};
  if (opts) o = *opts;
  RenderPlan p;
  int rc = render_check(ctx, views, n_views, out_dev, o, p);
  if (rc) return rc;

  CVX_HIP(hipSetDevice(ctx->device));
  if (ctx->staged_pending) {
    CVX_HIP(hipEventSynchronize(ctx->staged));
    ctx->staged_pending = false;
  }
  if ((size_t)n_views > ctx->stage_cap) {
    CVX_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->d_stage) (void)hipFree(ctx->d_stage);
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    ctx->d_stage = ctx->h_stage = nullptr;
    ctx->stage_cap = 0;
    const size_t bytes = sizeof(CastHeader) + sizeof(DView) * (size_t)n_views;
    CVX_HIP(hipMalloc(&ctx->d_stage, bytes));
    CVX_HIP(hipHostMalloc(&ctx->h_stage, bytes, 0));
    ctx->stage_cap = (size_t)n_views;
    drop_graph(ctx);
  }
  uint8_t* h = (uint8_t*)ctx->h_stage;
  uint8_t* d = (uint8_t*)ctx->d_stage;
  const RenderStage st{(DView*)(h + sizeof(CastHeader)), (CastHeader*)h,
                       (DView*)(d + sizeof(CastHeader)), (CastHeader*)d,
                       ctx->staged,                      &ctx->staged_pending,
                       true,                             ""};
  return render_launch(ctx, views, n_views, out_dev, o, p, st);
}

int cvx_render_noalloc(cvx_ctx* ctx, const cvx_view* views, int n_views, void* out_dev,
                       const cvx_render_opts* opts) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  cvx_render_opts o{};
  if (opts) o = *opts;
  if (n_views > CVX_NOALLOC_MAX_VIEWS)
    return fail(ctx, CVX_ERR_INVALID_ARG,
                "n_views " + std::to_string(n_views) + " exceeds CVX_NOALLOC_MAX_VIEWS (" +
                    std::to_string(CVX_NOALLOC_MAX_VIEWS) + ")");
  if (o.use_graph)
    return fail(ctx, CVX_ERR_INVALID_ARG, "cvx_render_noalloc takes no graph (use_graph = 0)");
  RenderPlan p;
  int rc = render_check(ctx, views, n_views, out_dev, o, p);
  if (rc) return rc;
  if (!ctx->d_scratch || !ctx->h_scratch)
    return fail(ctx, CVX_ERR_HIP, "the device scratch array was not found at cvx_create");
  CVX_HIP(hipSetDevice(ctx->device));
  // the previous call's copy out of the host staging must be done
  if (ctx->scratch_pending) {
    CVX_HIP(hipEventSynchronize(ctx->scratch_staged));
    ctx->scratch_pending = false;
  }
  uint8_t* h = (uint8_t*)ctx->h_scratch;
  uint8_t* d = (uint8_t*)ctx->d_scratch;
  const RenderStage st{(DView*)(h + sizeof(CastHeader)), (CastHeader*)h,
                       (DView*)(d + sizeof(CastHeader)), (CastHeader*)d,
                       ctx->scratch_staged,              &ctx->scratch_pending,
                       false,
                       "cvx_render_noalloc renders whole chords (chord_pieces 1): merging "
                       "pieces needs a buffer"};
  return render_launch(ctx, views, n_views, out_dev, o, p, st);
}

int cvx_pool_nodes(cvx_ctx* ctx, int canvas_id, uint64_t* n_nodes) {
  if (!ctx || !n_nodes) return CVX_ERR_INVALID_ARG;
  if (canvas_id < 0 || canvas_id >= CVX_MAX_CANVASES)
    return fail(ctx, CVX_ERR_INVALID_ARG, "canvas_id out of range");
  if (!ctx->canvases[canvas_id].present) return fail(ctx, CVX_ERR_NOT_FOUND, "no pool under canvas_id");
  *n_nodes = ctx->canvases[canvas_id].n_nodes;
  return CVX_OK;
}

int cvx_read_records(cvx_ctx* ctx, int canvas_id, uint64_t first, uint64_t count, uint32_t* out) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  if (canvas_id < 0 || canvas_id >= CVX_MAX_CANVASES)
    return fail(ctx, CVX_ERR_INVALID_ARG, "canvas_id out of range");
  const DevCanvas& c = ctx->canvases[canvas_id];
  if (!c.present) return fail(ctx, CVX_ERR_NOT_FOUND, "no pool under canvas_id");
  if (first > c.n_nodes || count > c.n_nodes - first || (count && !out))
    return fail(ctx, CVX_ERR_INVALID_ARG, "record range outside the pool");
  if (!count) return CVX_OK;
  CVX_HIP(hipSetDevice(ctx->device));
  CVX_HIP(hipStreamSynchronize(ctx->stream));
  CVX_HIP(hipMemcpy(out, (const uint8_t*)c.rec + first * 16, count * 16, hipMemcpyDeviceToHost));
  return CVX_OK;
}

namespace {

// The checks cvx_upload_pool makes on a leaf record.
bool leaf_ok(const void* payloads, uint64_t i, uint32_t fmt) {
  if (fmt == CVX_LEAF_RGBA8_F16) {
    uint16_t h;
    std::memcpy(&h, (const uint8_t*)payloads + i * 8 + 4, 2);
    const bool negative = (h & 0x8000u) && (h & 0x7fffu);
    const bool non_finite = (h & 0x7c00u) == 0x7c00u;
    return !negative && !non_finite;
  }
  double v[4];
  std::memcpy(v, (const uint8_t*)payloads + i * 32, 32);
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]) &&
         std::isfinite(v[3]) && v[3] >= 0.0;
}

// Host mirror of the record words x, from the device records.
int ensure_mirror(cvx_ctx* ctx, DevCanvas& c) {
  if (c.mirror_ready) return CVX_OK;
  c.mirror.assign(c.n_nodes, CVX_FREE);
  uint32_t* packed = nullptr;
  CVX_HIP(hipMalloc((void**)&packed, std::max<uint64_t>(c.n_nodes, 1) * 4));
  int le = cvx::launch_extract_x(ctx->stream, c.rec, c.n_nodes, packed);
  hipError_t e = (hipError_t)le;
  if (e == hipSuccess)
    e = hipMemcpyAsync(c.mirror.data(), packed, c.n_nodes * 4, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(packed);
  if (e != hipSuccess) return hip_fail(ctx, e, "reading the pool records back");
  c.leaves_at_depth.assign(64, 0);
  c.n_refined = 0;
  for (uint32_t x : c.mirror) {
    if (x == CVX_FREE) continue;
    if (x & 1u)
      ++c.leaves_at_depth[(x >> 1) & 63u];
    else
      ++c.n_refined;
  }
  c.free_groups.clear();
  c.mirror_ready = true;
  return CVX_OK;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// The edits of cvx_edit_pool on a present canvas (also the splits of a
// stroke step).
int edit_impl(cvx_ctx* ctx, DevCanvas& c, const cvx_edit* edits, uint32_t n_edits,
              const void* payloads, uint64_t n_payloads, uint32_t* first_child_out) {
  if (n_edits && !edits) return fail(ctx, CVX_ERR_INVALID_ARG, "edits is NULL");
  if (n_payloads && !payloads) return fail(ctx, CVX_ERR_INVALID_ARG, "payloads is NULL");
  CVX_HIP(hipSetDevice(ctx->device));
  int rc = ensure_mirror(ctx, c);
  if (rc) return rc;
  const uint32_t fmt = c.desc.leaf_format;
  const uint32_t lb = leaf_bytes(fmt);

  // ---- validate and apply to the mirror, with an undo log
  std::vector<std::pair<uint32_t, uint32_t>> undo;  // (node, old x)
  const std::vector<uint32_t> free0 = c.free_groups;
  const std::vector<uint64_t> depth0 = c.leaves_at_depth;
  const uint64_t refined0 = c.n_refined;
  uint64_t n_cur = c.n_nodes;
  std::vector<uint32_t> touched;                   // nodes whose record word changes
  std::vector<std::pair<uint32_t, uint64_t>> paint;  // (node, payload index), in order
  std::unordered_map<uint32_t, uint32_t> changed;   // refined or coarsened node -> depth
  auto set_x = [&](uint32_t i, uint32_t x) {
    undo.emplace_back(i, c.mirror[i]);
    c.mirror[i] = x;
    touched.push_back(i);
  };
  auto rollback = [&](int code, const std::string& m) {
    for (size_t j = undo.size(); j-- > 0;) c.mirror[undo[j].first] = undo[j].second;
    c.mirror.resize(c.n_nodes);
    c.free_groups = free0;
    c.leaves_at_depth = depth0;
    c.n_refined = refined0;
    return fail(ctx, code, m);
  };
  for (uint32_t e = 0; e < n_edits; ++e) {
    const cvx_edit& ed = edits[e];
    auto at = [e](const char* m) { return "edit " + std::to_string(e) + ": " + m; };
    if (first_child_out) first_child_out[e] = CVX_NONE_ID;
    if (ed.node >= n_cur) return rollback(CVX_ERR_INVALID_ARG, at("node out of range"));
    const uint32_t x = c.mirror[ed.node];
    if (x == CVX_FREE) return rollback(CVX_ERR_INVALID_ARG, at("node is not in the tree"));
    const bool leaf = (x & 1u) != 0;
    const uint32_t np = ed.op == CVX_EDIT_REFINE ? 8u : 1u;
    if (ed.op > CVX_EDIT_COARSEN) return rollback(CVX_ERR_INVALID_ARG, at("unknown op"));
    if (ed.first_payload > n_payloads || n_payloads - ed.first_payload < np)
      return rollback(CVX_ERR_INVALID_ARG, at("payload index out of range"));
    for (uint32_t j = 0; j < np; ++j)
      if (!leaf_ok(payloads, ed.first_payload + j, fmt))
        return rollback(CVX_ERR_INVALID_ARG, at("payload not finite or kappa < 0"));
    if (ed.op == CVX_EDIT_PAINT) {
      if (!leaf) return rollback(CVX_ERR_INVALID_ARG, at("PAINT needs a leaf"));
      paint.emplace_back(ed.node, ed.first_payload);
    } else if (ed.op == CVX_EDIT_REFINE) {
      if (!leaf) return rollback(CVX_ERR_INVALID_ARG, at("REFINE needs a leaf"));
      const uint32_t d = (x >> 1) & 63u;
      if (d + 1 > c.desc.max_depth)
        return rollback(CVX_ERR_INVALID_ARG, at("REFINE beyond the canvas max_depth"));
      uint64_t g;
      if (!c.free_groups.empty()) {
        g = c.free_groups.back();
        c.free_groups.pop_back();
      } else {
        g = (n_cur + 7) & ~7ull;
        if (g + 8 > (uint64_t)CVX_LEAF_BIT)
          return rollback(CVX_ERR_INVALID_ARG, at("pool would exceed 2^31 nodes"));
        c.mirror.resize(g + 8, CVX_FREE);
        n_cur = g + 8;
      }
      set_x(ed.node, (uint32_t)g);
      for (uint32_t o = 0; o < 8; ++o) {
        set_x((uint32_t)g + o, 1u | ((d + 1) << 1));
        paint.emplace_back((uint32_t)g + o, ed.first_payload + o);
        changed.erase((uint32_t)g + o);  // new children: covered by their parent
      }
      changed[ed.node] = d;
      --c.leaves_at_depth[d];
      c.leaves_at_depth[d + 1] += 8;
      ++c.n_refined;
      if (first_child_out) first_child_out[e] = (uint32_t)g;
    } else {
      if (leaf) return rollback(CVX_ERR_INVALID_ARG, at("COARSEN needs a refined node"));
      const uint32_t g = x;
      uint32_t dc = 0;
      for (uint32_t o = 0; o < 8; ++o) {
        const uint32_t cx = c.mirror[g + o];
        if (cx == CVX_FREE || !(cx & 1u))
          return rollback(CVX_ERR_INVALID_ARG, at("COARSEN needs 8 leaf children"));
        dc = (cx >> 1) & 63u;
      }
      set_x(ed.node, 1u | ((dc - 1) << 1));
      for (uint32_t o = 0; o < 8; ++o) {
        set_x(g + o, CVX_FREE);
        changed.erase(g + o);            // no longer in the tree
      }
      changed[ed.node] = dc - 1;
      c.free_groups.push_back(g);
      c.leaves_at_depth[dc] -= 8;
      ++c.leaves_at_depth[dc - 1];
      --c.n_refined;
      paint.emplace_back(ed.node, ed.first_payload);
    }
  }

  // ---- device: grow, scatter records and payloads, rebuild G_3 and the table
  auto device_fail = [&](hipError_t e, const char* where) {
    // the device may be partly updated: mark the mirror stale so the next
    // edit reads the device state back
    c.mirror_ready = false;
    c.mirror.clear();
    return hip_fail(ctx, e, where);
  };
  if (n_cur > c.cap_nodes) {
    uint64_t cap = std::max<uint64_t>(n_cur, std::min<uint64_t>(2 * c.cap_nodes, CVX_LEAF_BIT));
    size_t free_b = 0, total_b = 0;
    CVX_HIP(hipMemGetInfo(&free_b, &total_b));
    if (cap * (16 + lb) + (64ull << 20) > free_b) {
      cap = n_cur;
      if (cap * (16 + lb) + (64ull << 20) > free_b)
        return rollback(CVX_ERR_OOM, "growing the pool needs more device memory");
    }
    void *nrec = nullptr, *npay = nullptr;
    hipError_t e = hipMalloc(&nrec, cap * 16);
    if (e == hipSuccess) e = hipMalloc(&npay, cap * lb);
    if (e != hipSuccess) {
      if (nrec) (void)hipFree(nrec);
      return e == hipErrorOutOfMemory ? rollback(CVX_ERR_OOM, "device allocation failed")
                                      : rollback(CVX_ERR_HIP, "hipMalloc while growing the pool");
    }
    e = hipMemsetAsync(nrec, 0xff, cap * 16, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(nrec, c.rec, c.n_nodes * 16, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(npay, c.pay, c.n_nodes * lb, hipMemcpyDeviceToDevice, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
      (void)hipFree(nrec);
      (void)hipFree(npay);
      return device_fail(e, "growing the pool");
    }
    (void)hipFree(c.rec);
    (void)hipFree(c.pay);
    c.rec = nrec;
    c.pay = npay;
    c.bytes += (cap - c.cap_nodes) * (16 + lb);
    c.cap_nodes = cap;
  }
  c.n_nodes = n_cur;

  // last record word and last payload per node
  std::sort(touched.begin(), touched.end());
  touched.erase(std::unique(touched.begin(), touched.end()), touched.end());
  std::vector<uint32_t> xs(touched.size());
  for (size_t j = 0; j < touched.size(); ++j) xs[j] = c.mirror[touched[j]];
  std::vector<std::pair<uint32_t, uint64_t>> last;
  {
    std::vector<std::pair<uint32_t, uint64_t>> tmp;
    tmp.reserve(paint.size());
    for (size_t j = 0; j < paint.size(); ++j) tmp.emplace_back(paint[j].first, j);
    std::stable_sort(tmp.begin(), tmp.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    for (size_t j = 0; j < tmp.size(); ++j)
      if (j + 1 == tmp.size() || tmp[j + 1].first != tmp[j].first)
        last.emplace_back(tmp[j].first, paint[tmp[j].second].second);
  }
  std::vector<uint32_t> pay_ids(last.size());
  std::vector<uint8_t> pay_src(last.size() * lb);
  for (size_t j = 0; j < last.size(); ++j) {
    pay_ids[j] = last[j].first;
    std::memcpy(pay_src.data() + j * lb, (const uint8_t*)payloads + last[j].second * lb, lb);
  }
  const uint32_t R = c.desc.R;
  uint32_t depth = 0;
  for (uint32_t d = 0; d < 64; ++d)
    if (c.leaves_at_depth[d]) depth = d;
  std::vector<uint32_t> ch_ids, ch_depth;
  for (const auto& kv : changed) {
    ch_ids.push_back(kv.first);
    ch_depth.push_back(kv.second);
  }

  DevBuf b_ids, b_xs, b_pids, b_psrc, b_order, b_count, b_ch, b_chd, b_roots, b_rootd;
  hipError_t e = hipSuccess;
  const char* where = "";
#define STEP(call)                      \
  if (e == hipSuccess) {                \
    e = (call);                         \
    if (e != hipSuccess) where = #call; \
  }
  const uint64_t n_changed = ch_ids.size();
  STEP(hipMalloc(&b_ids.p, std::max<size_t>(touched.size(), 1) * 4));
  STEP(hipMalloc(&b_xs.p, std::max<size_t>(touched.size(), 1) * 4));
  STEP(hipMalloc(&b_pids.p, std::max<size_t>(pay_ids.size(), 1) * 4));
  STEP(hipMalloc(&b_psrc.p, std::max<size_t>(pay_src.size(), 8)));
  STEP(hipMalloc(&b_ch.p, std::max<uint64_t>(n_changed, 1) * 4));
  STEP(hipMalloc(&b_chd.p, std::max<uint64_t>(n_changed, 1) * 4));
  STEP(hipMalloc(&b_roots.p, std::max<uint64_t>(7 * n_changed, 1) * 4));
  STEP(hipMalloc(&b_rootd.p, std::max<uint64_t>(7 * n_changed, 1) * 4));
  STEP(hipMalloc(&b_count.p, 4));
  if (e == hipSuccess && c.mark_cap < c.n_nodes) {
    // per-node visit marks of the link rebuild (epochs), grown with the pool
    if (c.mark) (void)hipFree(c.mark);
    c.mark = nullptr;
    c.mark_cap = 0;
    STEP(hipMalloc((void**)&c.mark, c.cap_nodes * 4));
    STEP(hipMemsetAsync(c.mark, 0, c.cap_nodes * 4, ctx->stream));
    if (e == hipSuccess) c.mark_cap = c.cap_nodes;
  }
  if (e != hipSuccess) return device_fail(e, where);
  if (!touched.empty()) {
    STEP(hipMemcpyAsync(b_ids.p, touched.data(), touched.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    STEP(hipMemcpyAsync(b_xs.p, xs.data(), xs.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    if (e == hipSuccess) {
      int le = cvx::launch_scatter_records(ctx->stream, (const uint32_t*)b_ids.p,
                                           (const uint32_t*)b_xs.p, touched.size(), c.rec);
      if (le != hipSuccess) { e = (hipError_t)le; where = "k_scatter_records"; }
    }
  }
  if (!pay_ids.empty()) {
    STEP(hipMemcpyAsync(b_pids.p, pay_ids.data(), pay_ids.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    STEP(hipMemcpyAsync(b_psrc.p, pay_src.data(), pay_src.size(), hipMemcpyHostToDevice, ctx->stream));
    if (e == hipSuccess) {
      int le = cvx::launch_scatter_payloads(ctx->stream, (const uint32_t*)b_pids.p, b_psrc.p,
                                            pay_ids.size(), lb, c.pay);
      if (le != hipSuccess) { e = (hipError_t)le; where = "k_scatter_payloads"; }
    }
  }
  // G_3 below the changed regions (Sec. 4.1.2), on the final records: the
  // roots of the regions come from the device, then the links are derived
  // level by level as at upload, each level's frontier being the refined
  // children reached from the level above plus the region roots of that depth
  std::map<uint32_t, std::vector<uint32_t>> roots_at;
  uint64_t n_roots = 0;
  if (n_changed) {
    const uint32_t zero = 0;
    STEP(hipMemcpyAsync(b_ch.p, ch_ids.data(), n_changed * 4, hipMemcpyHostToDevice, ctx->stream));
    STEP(hipMemcpyAsync(b_chd.p, ch_depth.data(), n_changed * 4, hipMemcpyHostToDevice, ctx->stream));
    STEP(hipMemcpyAsync(b_count.p, &zero, 4, hipMemcpyHostToDevice, ctx->stream));
    if (e == hipSuccess) {
      int le = cvx::launch_dirty_roots(ctx->stream, (const uint32_t*)b_ch.p, (const uint32_t*)b_chd.p,
                                       n_changed, c.rec, R, (uint32_t*)b_roots.p,
                                       (uint32_t*)b_rootd.p, (uint32_t*)b_count.p, c.n_nodes);
      if (le != hipSuccess) { e = (hipError_t)le; where = "k_dirty_roots"; }
    }
    uint32_t cnt = 0;
    STEP(hipMemcpyAsync(&cnt, b_count.p, 4, hipMemcpyDeviceToHost, ctx->stream));
    STEP(hipStreamSynchronize(ctx->stream));
    if (e == hipSuccess && cnt > 7 * n_changed) { e = hipErrorUnknown; where = "region roots overflow"; }
    std::vector<uint32_t> rid(cnt), rd(cnt);
    if (cnt) {
      STEP(hipMemcpy(rid.data(), b_roots.p, cnt * 4, hipMemcpyDeviceToHost));
      STEP(hipMemcpy(rd.data(), b_rootd.p, cnt * 4, hipMemcpyDeviceToHost));
    }
    for (uint32_t j = 0; e == hipSuccess && j < cnt; ++j) roots_at[rd[j]].push_back(rid[j]);
    for (auto& kv : roots_at) {
      std::sort(kv.second.begin(), kv.second.end());
      kv.second.erase(std::unique(kv.second.begin(), kv.second.end()), kv.second.end());
      n_roots += kv.second.size();
    }
  }
  if (e == hipSuccess && !roots_at.empty()) {
    const uint64_t cap = c.n_refined + n_roots;
    STEP(hipMalloc(&b_order.p, std::max<uint64_t>(cap, 1) * 4));
    const uint32_t epoch = ++c.epoch;  // marks hold 0 or an earlier epoch
    uint64_t lo = 0, hi = 0;
    auto it = roots_at.begin();
    for (uint32_t level = it->first; e == hipSuccess; ++level) {
      if (it != roots_at.end() && it->first == level) {
        if (hi + it->second.size() > cap) { e = hipErrorUnknown; where = "link frontier overflow"; break; }
        STEP(hipMemcpyAsync((uint32_t*)b_order.p + hi, it->second.data(), it->second.size() * 4,
                            hipMemcpyHostToDevice, ctx->stream));
        hi += it->second.size();
        ++it;
      }
      if (hi == lo) {
        if (it == roots_at.end()) break;
        continue;
      }
      const uint32_t h32 = (uint32_t)hi;
      STEP(hipMemcpyAsync(b_count.p, &h32, 4, hipMemcpyHostToDevice, ctx->stream));
      if (e != hipSuccess) break;
      int le = cvx::launch_links_level(ctx->stream, (const uint32_t*)b_order.p + lo, hi - lo, level,
                                       c.rec, R, (uint32_t*)b_order.p, (uint32_t*)b_count.p,
                                       c.n_nodes, c.mark, epoch);
      if (le != hipSuccess) { e = (hipError_t)le; where = "k_links_level"; break; }
      uint32_t cnt = 0;
      STEP(hipMemcpyAsync(&cnt, b_count.p, 4, hipMemcpyDeviceToHost, ctx->stream));
      STEP(hipStreamSynchronize(ctx->stream));
      if (e != hipSuccess) break;
      if (cnt > cap) { e = hipErrorUnknown; where = "link frontier overflow"; break; }
      lo = hi;
      hi = cnt;
    }
  }
  // top-level table for the new depth
  const uint32_t L = cvx::top_table_depth(R, depth);
  if (e == hipSuccess && L != c.top_depth) {
    if (c.top) (void)hipFree(c.top);
    c.top = nullptr;
    c.top_depth = 0;
    if (L) {
      const uint64_t side = (uint64_t)R << L;
      STEP(hipMalloc((void**)&c.top, side * side * side * 4));
      if (e == hipSuccess) c.top_depth = L;
    }
  }
  if (e == hipSuccess && c.top_depth) {
    int le = cvx::launch_top_table(ctx->stream, c.rec, c.n_nodes, R, c.top_depth, c.top);
    if (le != hipSuccess) { e = (hipError_t)le; where = "k_top_table"; }
  }
  STEP(hipStreamSynchronize(ctx->stream));
#undef STEP
  if (e != hipSuccess) return device_fail(e, where);
  c.depth = depth;
  return CVX_OK;
}

}  // namespace

int cvx_edit_pool(cvx_ctx* ctx, int canvas_id, const cvx_edit* edits, uint32_t n_edits,
                  const void* payloads, uint64_t n_payloads, uint32_t* first_child_out) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  if (canvas_id < 0 || canvas_id >= CVX_MAX_CANVASES)
    return fail(ctx, CVX_ERR_INVALID_ARG, "canvas_id out of range");
  DevCanvas& c = ctx->canvases[canvas_id];
  if (!c.present) return fail(ctx, CVX_ERR_NOT_FOUND, "no pool under canvas_id");
  c.stroke = cvx::StrokeState();
  return edit_impl(ctx, c, edits, n_edits, payloads, n_payloads, first_child_out);
}

int cvx_read_payloads(cvx_ctx* ctx, int canvas_id, uint64_t first, uint64_t count, void* out) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  if (canvas_id < 0 || canvas_id >= CVX_MAX_CANVASES)
    return fail(ctx, CVX_ERR_INVALID_ARG, "canvas_id out of range");
  const DevCanvas& c = ctx->canvases[canvas_id];
  if (!c.present) return fail(ctx, CVX_ERR_NOT_FOUND, "no pool under canvas_id");
  if (first > c.n_nodes || count > c.n_nodes - first || (count && !out))
    return fail(ctx, CVX_ERR_INVALID_ARG, "payload range outside the pool");
  if (!count) return CVX_OK;
  const uint64_t lb = leaf_bytes(c.desc.leaf_format);
  CVX_HIP(hipSetDevice(ctx->device));
  CVX_HIP(hipStreamSynchronize(ctx->stream));
  CVX_HIP(hipMemcpy(out, (const uint8_t*)c.pay + first * lb, count * lb, hipMemcpyDeviceToHost));
  return CVX_OK;
}

namespace {

// IEEE half <-> float, round to nearest even (host side of the leaf format).
float half_to_float(uint16_t h) {
  const uint32_t sign = (uint32_t)(h & 0x8000u) << 16, ex = (h >> 10) & 0x1fu, man = h & 0x3ffu;
  float v;
  if (ex == 0) {
    v = std::ldexp((float)man, -24);
    return sign ? -v : v;
  }
  const uint32_t bits = ex == 31 ? (sign | 0x7f800000u | (man << 13))
                                 : (sign | ((ex + 112u) << 23) | (man << 13));
  std::memcpy(&v, &bits, 4);
  return v;
}

uint16_t float_to_half(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint32_t sign = (x >> 16) & 0x8000u, ax = x & 0x7fffffffu;
  if (ax >= 0x7f800000u) return (uint16_t)(sign | (ax > 0x7f800000u ? 0x7e00u : 0x7c00u));
  if (ax >= 0x477ff000u) return (uint16_t)(sign | 0x7c00u);  // 65520 and up round to inf
  if (ax < 0x38800000u) {                                     // below 2^-14: subnormal
    float a;
    std::memcpy(&a, &ax, 4);
    return (uint16_t)(sign | (uint32_t)std::nearbyint(a * 16777216.0f));
  }
  uint32_t h = (((ax >> 23) - 112u) << 10) | ((ax & 0x7fffffu) >> 13);
  const uint32_t rem = ax & 0x1fffu;
  if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;
  return (uint16_t)(sign | h);
}

// Payload of the children of a split leaf: same colour, half the optical
// depth per edge (A recomputed from it).
void child_payload(const uint8_t* parent, uint32_t fmt, uint8_t* child) {
  if (fmt == CVX_LEAF_F64) {
    double q[4];
    std::memcpy(q, parent, 32);
    q[3] = q[3] * 0.5;
    std::memcpy(child, q, 32);
    return;
  }
  uint16_t h;
  std::memcpy(&h, parent + 4, 2);
  const uint16_t hc = float_to_half(half_to_float(h) * 0.5f);
  const double kc = (double)half_to_float(hc);
  std::memcpy(child, parent, 8);
  child[3] = (uint8_t)std::lrint(255.0 * (1.0 - std::exp(-kc)));
  std::memcpy(child + 4, &hc, 2);
  child[6] = child[7] = 0;
}

// One walk of the stroke from a frontier (nullptr: the root array) down to
// the leaves, level by level on the GPU; the leaves still waiting for a split
// are appended to c.stroke.pending with their payloads from before the stroke.
int stroke_walk(cvx_ctx* ctx, DevCanvas& c, const std::vector<cvx::StrokeItem>* start,
                uint32_t merge = 0) {
  cvx::StrokeState& st = c.stroke;
  const uint32_t lb = leaf_bytes(c.desc.leaf_format);
  const uint32_t R = c.desc.R;
  uint64_t n = start ? start->size() : (uint64_t)R * R * R;
  if (!n) return CVX_OK;
  DevBuf b_stamps, b_cur, b_count;
  hipError_t e = hipSuccess;
  const char* where = "";
#define STEP(call)                      \
  if (e == hipSuccess) {                \
    e = (call);                         \
    if (e != hipSuccess) where = #call; \
  }
  STEP(hipMalloc(&b_stamps.p, st.stamps.size() * 8));
  STEP(hipMemcpyAsync(b_stamps.p, st.stamps.data(), st.stamps.size() * 8, hipMemcpyHostToDevice,
                      ctx->stream));
  STEP(hipMalloc(&b_count.p, 8));
  if (start) {
    STEP(hipMalloc(&b_cur.p, n * sizeof(cvx::StrokeItem)));
    STEP(hipMemcpyAsync(b_cur.p, start->data(), n * sizeof(cvx::StrokeItem),
                        hipMemcpyHostToDevice, ctx->stream));
  }
  for (uint32_t level = 0; e == hipSuccess && n; ++level) {
    if (n > 0x1fffffffull) { e = hipErrorUnknown; where = "stroke frontier too large"; break; }
    DevBuf b_next, b_pend, b_ppay;
    STEP(hipMalloc(&b_next.p, 8 * n * sizeof(cvx::StrokeItem)));
    STEP(hipMalloc(&b_pend.p, n * sizeof(cvx::StrokeItem)));
    STEP(hipMalloc(&b_ppay.p, n * lb));
    STEP(hipMemsetAsync(b_count.p, 0, 8, ctx->stream));
    if (e != hipSuccess) break;
    uint32_t* cnt = (uint32_t*)b_count.p;
    int le = cvx::launch_stroke_visit(ctx->stream, (const cvx::StrokeItem*)b_cur.p, (uint32_t)n,
                                      st.args, b_stamps.p, c.rec, c.pay, c.n_nodes,
                                      (cvx::StrokeItem*)b_next.p, cnt, (uint32_t)(8 * n),
                                      (cvx::StrokeItem*)b_pend.p, b_ppay.p, cnt + 1, (uint32_t)n,
                                      merge);
    if (le != hipSuccess) { e = (hipError_t)le; where = "k_stroke_visit"; break; }
    uint32_t h[2] = {0, 0};
    STEP(hipMemcpyAsync(h, b_count.p, 8, hipMemcpyDeviceToHost, ctx->stream));
    STEP(hipStreamSynchronize(ctx->stream));
    if (e != hipSuccess) break;
    if (h[0] > 8 * n || h[1] > n) { e = hipErrorUnknown; where = "stroke frontier overflow"; break; }
    if (h[1]) {
      const size_t p0 = st.pending.size();
      st.pending.resize(p0 + h[1]);
      st.pending_pay.resize((p0 + h[1]) * lb);
      STEP(hipMemcpy(st.pending.data() + p0, b_pend.p, h[1] * sizeof(cvx::StrokeItem),
                     hipMemcpyDeviceToHost));
      STEP(hipMemcpy(st.pending_pay.data() + p0 * lb, b_ppay.p, (size_t)h[1] * lb,
                     hipMemcpyDeviceToHost));
    }
    std::swap(b_cur.p, b_next.p);
    n = h[0];
  }
#undef STEP
  if (e != hipSuccess) return hip_fail(ctx, e, where);
  return CVX_OK;
}

// Payload of the leaf that replaces 8 identical children: same colour, twice
// the optical depth per edge (A recomputed).  False when the half kappa
// would overflow.
bool parent_payload(const uint8_t* child, uint32_t fmt, uint8_t* parent) {
  if (fmt == CVX_LEAF_F64) {
    double q[4];
    std::memcpy(q, child, 32);
    q[3] = q[3] * 2.0;
    std::memcpy(parent, q, 32);
    return std::isfinite(q[3]);
  }
  uint16_t h;
  std::memcpy(&h, child + 4, 2);
  const double kp = (double)half_to_float(h) * 2.0;
  if (kp > 65504.0) return false;
  const uint16_t hp = float_to_half((float)kp);
  std::memcpy(parent, child, 8);
  parent[3] = (uint8_t)std::lrint(255.0 * (1.0 - std::exp(-kp)));
  std::memcpy(parent + 4, &hp, 2);
  parent[6] = parent[7] = 0;
  return true;
}

// When a coarsening stroke has no split left, the next steps merge: the
// walk lists the cells that can merge now.
int stroke_enter_merge(cvx_ctx* ctx, DevCanvas& c) {
  cvx::StrokeState& st = c.stroke;
  if (!st.pending.empty() || !st.coarsen || st.merging) return CVX_OK;
  st.merging = true;
  return stroke_walk(ctx, c, nullptr, 1);
}

// One level of merges: COARSEN edits for the listed cells, then the walk for
// the next level.
int stroke_merge_step(cvx_ctx* ctx, DevCanvas& c) {
  cvx::StrokeState& st = c.stroke;
  const uint32_t fmt = c.desc.leaf_format, lb = leaf_bytes(fmt);
  std::vector<uint32_t> nodes;
  std::vector<uint8_t> pays;
  for (size_t i = 0; i < st.pending.size(); ++i) {
    uint8_t pp[32];
    if (!parent_payload(st.pending_pay.data() + i * lb, fmt, pp)) continue;
    nodes.push_back(st.pending[i].node);
    pays.insert(pays.end(), pp, pp + lb);
  }
  std::vector<uint32_t> ord(nodes.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = (uint32_t)i;
  std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return nodes[a] < nodes[b]; });
  std::vector<cvx_edit> edits(nodes.size());
  for (size_t i = 0; i < ord.size(); ++i) {
    edits[i].op = CVX_EDIT_COARSEN;
    edits[i].node = nodes[ord[i]];
    edits[i].first_payload = ord[i];
  }
  st.pending.clear();
  st.pending_pay.clear();
  if (!edits.empty()) {
    int rc = edit_impl(ctx, c, edits.data(), (uint32_t)edits.size(), pays.data(),
                       (uint64_t)nodes.size(), nullptr);
    if (rc != CVX_OK) return rc;
    // a merge that overflowed the half kappa stays refined; only merged cells
    // can make their parents mergeable, so walk again only after merges
    return stroke_walk(ctx, c, nullptr, 1);
  }
  return CVX_OK;
}

int stroke_step_impl(cvx_ctx* ctx, DevCanvas& c, uint64_t* pending) {
  cvx::StrokeState& st = c.stroke;
  if (!st.active || st.pending.empty()) {
    st = cvx::StrokeState();
    if (pending) *pending = 0;
    return CVX_OK;
  }
  if (st.merging) {
    int rc = stroke_merge_step(ctx, c);
    if (rc != CVX_OK || st.pending.empty()) st = cvx::StrokeState();
    if (pending) *pending = st.pending.size();
    return rc;
  }
  const uint32_t fmt = c.desc.leaf_format, lb = leaf_bytes(fmt);
  const size_t n = st.pending.size();
  if (n > 0xffffffffull / 8) {
    st = cvx::StrokeState();
    return fail(ctx, CVX_ERR_INVALID_ARG, "too many leaves waiting for a split");
  }
  // splits in ascending node order, so that the ids the children get do not
  // depend on the order in which the GPU appended the waiting leaves
  std::vector<uint32_t> ord(n);
  for (size_t i = 0; i < n; ++i) ord[i] = (uint32_t)i;
  std::sort(ord.begin(), ord.end(),
            [&](uint32_t a, uint32_t b) { return st.pending[a].node < st.pending[b].node; });
  std::vector<cvx_edit> edits(n);
  std::vector<uint8_t> pays(n * 8 * lb);
  for (size_t i = 0; i < n; ++i) {
    edits[i].op = CVX_EDIT_REFINE;
    edits[i].node = st.pending[ord[i]].node;
    edits[i].first_payload = 8 * (uint64_t)i;
    uint8_t cp[32];
    child_payload(st.pending_pay.data() + (size_t)ord[i] * lb, fmt, cp);
    for (uint32_t o = 0; o < 8; ++o) std::memcpy(pays.data() + (8 * i + o) * lb, cp, lb);
  }
  std::vector<uint32_t> first(n);
  int rc = edit_impl(ctx, c, edits.data(), (uint32_t)n, pays.data(), 8 * (uint64_t)n,
                     first.data());
  if (rc != CVX_OK) {
    st = cvx::StrokeState();
    return rc;
  }
  std::vector<cvx::StrokeItem> kids(8 * n);
  for (size_t i = 0; i < n; ++i) {
    const cvx::StrokeItem& p = st.pending[ord[i]];
    for (uint32_t o = 0; o < 8; ++o) {
      cvx::StrokeItem& k = kids[8 * i + o];
      k = cvx::StrokeItem{};
      k.node = first[i] + o;
      k.x = 2 * p.x + (o & 1u);
      k.y = 2 * p.y + ((o >> 1) & 1u);
      k.z = 2 * p.z + ((o >> 2) & 1u);
      k.depth = p.depth + 1;
    }
  }
  st.pending.clear();
  st.pending_pay.clear();
  rc = stroke_walk(ctx, c, &kids);
  if (rc == CVX_OK) rc = stroke_enter_merge(ctx, c);
  if (rc != CVX_OK) {
    st = cvx::StrokeState();
    return rc;
  }
  if (st.pending.empty()) st = cvx::StrokeState();
  if (pending) *pending = st.pending.size();
  return CVX_OK;
}

}  // namespace

int cvx_stroke_begin(cvx_ctx* ctx, int canvas_id, const cvx_stroke* stroke, const double* stamps,
                     uint32_t n_stamps, uint64_t* pending) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  if (canvas_id < 0 || canvas_id >= CVX_MAX_CANVASES)
    return fail(ctx, CVX_ERR_INVALID_ARG, "canvas_id out of range");
  DevCanvas& c = ctx->canvases[canvas_id];
  if (!c.present) return fail(ctx, CVX_ERR_NOT_FOUND, "no pool under canvas_id");
  if (!stroke) return fail(ctx, CVX_ERR_INVALID_ARG, "stroke is NULL");
  if (n_stamps < 1 || n_stamps > CVX_MAX_STAMPS || !stamps)
    return fail(ctx, CVX_ERR_INVALID_ARG, "n_stamps must be in [1, CVX_MAX_STAMPS]");
  for (int k = 0; k < 3; ++k)
    if (!(stroke->rgb[k] >= 0.0 && stroke->rgb[k] <= 1.0))
      return fail(ctx, CVX_ERR_INVALID_ARG, "stroke colour outside [0, 1]");
  if (!(std::isfinite(stroke->sigma) && stroke->sigma >= 0.0))
    return fail(ctx, CVX_ERR_INVALID_ARG, "stroke sigma must be finite and >= 0");
  if (!(std::isfinite(stroke->radius) && stroke->radius > 0.0))
    return fail(ctx, CVX_ERR_INVALID_ARG, "stroke radius must be finite and > 0");
  if (!(std::isfinite(stroke->k_refine) && stroke->k_refine > 0.0))
    return fail(ctx, CVX_ERR_INVALID_ARG, "stroke k_refine must be finite and > 0");
  if (stroke->coarsen > 1) return fail(ctx, CVX_ERR_INVALID_ARG, "stroke coarsen must be 0 or 1");
  for (uint64_t j = 0; j < 4ull * n_stamps; ++j)
    if (!std::isfinite(stamps[j]) || (j % 4 == 3 && stamps[j] < 0.0))
      return fail(ctx, CVX_ERR_INVALID_ARG,
                  "stamp " + std::to_string(j / 4) + " not finite or with r < 0");
  CVX_HIP(hipSetDevice(ctx->device));
  // a stroke still in progress is completed first (one level per step: at
  // most max_depth levels of splits and as many of merges)
  for (uint32_t guard = 0; c.stroke.active && guard <= 2 * CVX_MAX_DEPTH + 2; ++guard) {
    int rc = stroke_step_impl(ctx, c, nullptr);
    if (rc != CVX_OK) return rc;
  }
  CVX_HIP(hipStreamSynchronize(ctx->stream));
  cvx::StrokeState st;
  for (int k = 0; k < 3; ++k) {
    st.args.origin[k] = c.desc.origin[k];
    st.args.rgb[k] = stroke->rgb[k];
  }
  st.args.root_edge = c.desc.root_edge;
  st.args.sigma = stroke->sigma;
  st.args.radius = stroke->radius;
  st.args.hmin = stroke->radius / stroke->k_refine;
  st.args.R = c.desc.R;
  st.args.max_depth = c.desc.max_depth;
  st.args.fmt = c.desc.leaf_format;
  st.args.n_stamps = n_stamps;
  st.stamps.assign(stamps, stamps + 4ull * n_stamps);
  st.active = true;
  st.coarsen = stroke->coarsen != 0;
  c.stroke = std::move(st);
  int rc = stroke_walk(ctx, c, nullptr);
  if (rc == CVX_OK) rc = stroke_enter_merge(ctx, c);
  if (rc != CVX_OK) {
    c.stroke = cvx::StrokeState();
    return rc;
  }
  if (c.stroke.pending.empty()) c.stroke = cvx::StrokeState();
  if (pending) *pending = c.stroke.pending.size();
  return CVX_OK;
}

int cvx_stroke_step(cvx_ctx* ctx, int canvas_id, uint64_t* pending) {
  if (!ctx) return CVX_ERR_INVALID_ARG;
  ctx->err.clear();
  if (canvas_id < 0 || canvas_id >= CVX_MAX_CANVASES)
    return fail(ctx, CVX_ERR_INVALID_ARG, "canvas_id out of range");
  DevCanvas& c = ctx->canvases[canvas_id];
  if (!c.present) return fail(ctx, CVX_ERR_NOT_FOUND, "no pool under canvas_id");
  CVX_HIP(hipSetDevice(ctx->device));
  CVX_HIP(hipStreamSynchronize(ctx->stream));
  return stroke_step_impl(ctx, c, pending);
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
  // one untimed render (it also captures the graph), then reps timed ones
  auto time_candidate = [&](const cvx_render_opts& o, float& ms) -> int {
    int r = cvx_render(ctx, views, n_views, out_dev, &o);
    if (r != CVX_OK) return r;
    if ((he = hipEventRecord(e0, ctx->stream)) != hipSuccess)
      return hip_fail(ctx, he, "hipEventRecord");
    for (uint32_t i = 0; i < reps && r == CVX_OK; ++i) r = cvx_render(ctx, views, n_views, out_dev, &o);
    if (r != CVX_OK) return r;
    if ((he = hipEventRecord(e1, ctx->stream)) != hipSuccess ||
        (he = hipEventSynchronize(e1)) != hipSuccess ||
        (he = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
      return hip_fail(ctx, he, "timing a candidate");
    ms /= (float)reps;
    return CVX_OK;
  };
  auto record = [&](const cvx_render_opts& o, float ms) {
    if (count < max_results) {
      cvx_tune_result& x = results[count];
      x.tile_w = o.tile_w;
      x.tile_h = o.tile_h;
      x.wg_size = o.wg_size;
      x.workgroups = o.workgroups;
      x.ms = ms;
      x.top_lookup = o.top_lookup;
      x.single_queue = o.single_queue;
      x.rays_per_wave = o.rays_per_wave ? o.rays_per_wave : 64u;
      x.refill_min = o.rays_per_wave > 64u ? o.refill_min : 0u;
      x.chord_pieces = o.chord_pieces ? o.chord_pieces : 1u;
    }
    ++count;
    if (!have || ms < best_ms) {
      have = true;
      best_ms = ms;
      *best = o;
    }
  };
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
        o.rays_per_wave = 0;
        o.refill_min = 0;
        o.chord_pieces = 0;
        float ms = 0.0f;
        rc = time_candidate(o, ms);
        if (rc != CVX_OK) break;
        record(o, ms);
      }
    }
  }
  }
  }
  // lane refill on the fastest shape (FP32 renders only)
  if (rc == CVX_OK && have && b.variant == CVX_VARIANT_FP32_REBASED) {
    static const uint32_t kRpw[] = {128, 256};
    static const uint32_t kMin[] = {16, 32, 48};
    const cvx_render_opts shape = *best;
    for (uint32_t rpw : kRpw) {
      for (uint32_t mn : kMin) {
        if (rc != CVX_OK) break;
        cvx_render_opts o = shape;
        o.rays_per_wave = rpw;
        o.refill_min = mn;
        float ms = 0.0f;
        rc = time_candidate(o, ms);
        if (rc != CVX_OK) break;
        record(o, ms);
      }
    }
    // chord pieces on the same shape
    static const uint32_t kPieces[] = {2, 4, 8};
    for (uint32_t pc : kPieces) {
      if (rc != CVX_OK) break;
      cvx_render_opts o = shape;
      o.chord_pieces = pc;
      float ms = 0.0f;
      rc = time_candidate(o, ms);
      if (rc != CVX_OK) break;
      record(o, ms);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (n_results) *n_results = count;
  return rc;
}

}  // extern "C"

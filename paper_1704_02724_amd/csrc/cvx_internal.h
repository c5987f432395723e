// Internal declarations shared by the libcvx translation units.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cvx.h"

#define CVX_LEAF_BIT 0x80000000u
#define CVX_NONE 0xffffffffu
#define CVX_FREE 0xffffffffu  // record word x of a node that is not in the tree

namespace cvx {

// Breadth-first order of the reachable nodes, one range per level.
struct PoolPlan {
  std::vector<uint32_t> order;
  std::vector<uint64_t> level_off;  // level d is order[level_off[d], level_off[d+1])
  uint32_t depth = 0;               // deepest level present
};

int check_desc(const cvx_canvas_desc* d, std::string& msg);
int validate_pool(const cvx_canvas_desc* desc, const cvx_node* nodes, uint64_t n_nodes,
                  const void* leaves, uint64_t n_leaves, PoolPlan* plan, std::string& msg);
int validate_views(const cvx_view* views, int n_views, const cvx_canvas_desc* const* canvases,
                   int n_canvases, std::string& msg);

// Device node record (16 bytes), one per pool node, indexed like the input:
//   x: leaf -> 1 | depth << 1 ; refined -> index of the first child (multiple of 8, even)
//   y, z, w: outer-face neighbour on the x, y, z axis: the cell of the same
//            depth across the face of the parent that this child touches, or
//            the coarser leaf covering it; CVX_NONE outside the canvas or for roots.
// Payload (indexed by node id): RGBA8 + half kappa (uint2) or 4 doubles.
// A cell on the walk of a brush stroke: node id, integer coordinates at its
// depth (root array at depth 0), depth.
struct StrokeItem {
  uint32_t node, x, y, z, depth, pad0, pad1, pad2;
};

// One stroke in device-ready form (world units, as the canvas descriptor).
struct StrokeArgs {
  double origin[3];
  double root_edge;
  double rgb[3];
  double sigma, radius, hmin;  // hmin = radius / k_refine
  uint32_t R, max_depth, fmt, n_stamps;
};

// A stroke whose splits are still being applied, one level per step: its
// parameters and stamps, and the leaves waiting for a split with their
// payloads from before the stroke.
struct StrokeState {
  bool active = false;
  bool coarsen = false;  // merge uniform cells once the splits are done
  bool merging = false;  // pending holds cells to merge, not leaves to split
  StrokeArgs args{};
  std::vector<double> stamps;  // 4 per stamp: x, y, z, r
  std::vector<StrokeItem> pending;
  std::vector<uint8_t> pending_pay;
};

struct DevCanvas {
  bool present = false;
  cvx_canvas_desc desc{};
  uint64_t n_nodes = 0;
  uint32_t depth = 0;     // deepest level present
  void* rec = nullptr;    // uint4 per node
  void* pay = nullptr;    // uint2 or double4 per node
  uint32_t* top = nullptr;  // top-level table: node covering each cell of depth top_depth
  uint32_t top_depth = 0;   // 0: no table
  uint64_t bytes = 0;
  // pool edits: device capacity in nodes, and a host mirror of every record
  // word x (built on the first edit), the freed groups (LIFO) and the leaf
  // count per depth
  uint64_t cap_nodes = 0;
  bool mirror_ready = false;
  std::vector<uint32_t> mirror;
  std::vector<uint32_t> free_groups;
  std::vector<uint64_t> leaves_at_depth;
  uint64_t n_refined = 0;  // refined nodes in the tree
  uint32_t* mark = nullptr;  // per node: last edit call whose link rebuild visited it
  uint64_t mark_cap = 0;
  uint32_t epoch = 0;
  StrokeState stroke;
};

// Depth of the top-level table of a canvas: at most 6 levels and 2^18 cells,
// never below the deepest level present; 0 means no table.
inline uint32_t top_table_depth(uint32_t R, uint32_t depth) {
  uint32_t L = depth < 6 ? depth : 6;
  while (L > 0 && ((uint64_t)R << L) * ((uint64_t)R << L) * ((uint64_t)R << L) > (1ull << 18)) --L;
  return L;
}

// Per-view parameters in device memory (host computes them once per render).
struct DView {
  const void* rec;
  const void* pay;
  uint32_t R, fmt, max_depth, tiles_x;
  double o[3];          // eye in root-edge units
  double right[3], up[3], fwd[3];
  double tan_x, tan_y;
  double two_w, two_h;  // 2 / W and 2 / H, rounded once
  uint32_t W, H;
  uint64_t out_off;
  uint64_t first_tile;  // prefix sum of tile counts over the views
  float alpha_stop;
  uint32_t max_steps;
  uint32_t n_nodes;     // node ids at or above this are never loaded
  uint32_t top_depth;   // 0: ray starts descend from the root array
  const uint32_t* top;  // (R 2^top_depth)^3 node ids, x fastest
  // the leaf holding the eye when every ray of the view starts there (eye
  // inside the canvas, off every plane of the deepest grid), written on the
  // device before the cast; start_ok = 0: each ray locates its first leaf
  uint32_t start_ok, start_node, start_dep;
  uint32_t start_c[3];  // its integer coordinates at start_dep
  uint32_t pieces;      // chord pieces per ray (1: unsplit)
  float t_stop;         // 1 - alpha_stop, rounded once: the FP32 caster stops once T <= t_stop
};

// Work queues: the work items (tiles or 64-ray chunks) are split into
// CVX_NQ contiguous ranges, one per XCD (a workgroup runs on XCD
// blockIdx.x mod 8), so the tiles one XCD renders are neighbours and share
// its L2.  A wavefront drains its own range first, then the others in turn.
constexpr uint32_t CVX_NQ = 8;

struct alignas(128) QueueHead {
  uint32_t next;  // items taken from this range so far
  uint32_t pad[31];
};

// Launch-invariant header in device memory, so a captured graph can be
// replayed for any view set of the same launch shape.
struct CastHeader {
  uint64_t total_work;  // tiles (render) or 64-ray chunks (trace)
  uint64_t n_rays;      // trace mode: number of listed rays
  uint32_t n_views;
  uint32_t n_queues;        // 1 or CVX_NQ ranges in use
  uint32_t pad[26];
  QueueHead queue[CVX_NQ];  // reset by a kernel before each cast
};

struct CastArgs {
  const DView* views;
  CastHeader* hdr;
  void* out;
  const cvx_trace* trace_host;  // unused on device
  // trace mode
  const uint64_t* ray_ids;
  uint32_t max_leaves;
  uint32_t* leaf_ids;
  float* local_len;
  double* local_len64;
  uint32_t* n_leaves;
  uint32_t* flags;
  float* trace_rgba;
  double* end_point;
  uint64_t* stats;
  uint32_t tile_w, tile_h;
  uint32_t small_pools;  // every pool the views read has at most 2^28 nodes
  // FP32 render with lane refill when item_tiles > 1: a work item is up to
  // item_tiles tiles of one view, and waiting lanes take its next rays once
  // refill_min lanes of the wavefront wait
  uint32_t item_tiles;
  uint32_t refill_min;
  // FP32 render or trace of chord pieces when pieces > 1: a view with
  // pieces > 1 splits each ray's chord into that many consecutive pieces,
  // traced as separate work items; render pieces write (colour, T) to
  // split_tmp[pixel * pieces + piece] for the merge
  uint32_t pieces;
  void* split_tmp;
};

// kernel launchers (cvx_upload.hip, cvx_cast.hip); return a hipError_t value
int launch_top_table(void* stream, const void* rec, uint64_t n_nodes, uint32_t R, uint32_t L,
                     uint32_t* top);
int launch_extract_x(void* stream, const void* rec, uint64_t n, uint32_t* out);
int launch_scatter_records(void* stream, const uint32_t* ids, const uint32_t* xs, uint64_t n,
                           void* rec);
int launch_scatter_payloads(void* stream, const uint32_t* ids, const void* src, uint64_t n,
                            uint32_t leaf_bytes, void* pay);
int launch_links_level(void* stream, const uint32_t* frontier, uint64_t n, uint32_t level,
                       void* rec, uint32_t R, uint32_t* next, uint32_t* next_count,
                       uint64_t n_nodes, uint32_t* mark, uint32_t epoch);
int launch_dirty_roots(void* stream, const uint32_t* changed, const uint32_t* depth, uint64_t n,
                       const void* rec, uint32_t R, uint32_t* out, uint32_t* out_depth,
                       uint32_t* out_count, uint64_t n_nodes);
int launch_relayout_level(void* stream, const uint32_t* order, uint64_t begin, uint64_t end,
                          uint32_t level, const void* raw_nodes, const void* raw_leaves,
                          uint32_t fmt, void* rec, void* pay, uint32_t R);
int launch_cast(void* stream, uint32_t variant, bool trace, bool stats, bool out_f64,
                const CastArgs& a, uint32_t workgroups, uint32_t wg_size);
// the front-to-back merge of chord pieces into out (views with pieces > 1)
int launch_merge_pieces(void* stream, const DView* views, const CastHeader* hdr, uint32_t n_views,
                        const void* tmp, void* out, uint32_t stride);
// Scratch of the allocation-free render entry point: a CastHeader followed by
// CVX_NOALLOC_MAX_VIEWS view records, in a fixed device array of
// cvx_cast.hip.  scratch_address returns its address on the current device
// (looked up once per device; call with that device current).
constexpr size_t CVX_SCRATCH_BYTES = sizeof(CastHeader) + CVX_NOALLOC_MAX_VIEWS * sizeof(DView);
int scratch_address(int device, void** ptr);
// the shared first leaf of every view whose eye lies inside its canvas
int launch_view_starts(void* stream, DView* views, CastHeader* hdr, uint32_t enable);
// one level of a stroke's walk (cvx_stroke.hip); items == nullptr: the roots;
// merge = 1: find cells to merge instead of painting and splitting
int launch_stroke_visit(void* stream, const StrokeItem* items, uint32_t n, const StrokeArgs& a,
                        const void* stamps, const void* rec, void* pay, uint64_t n_nodes,
                        StrokeItem* next, uint32_t* next_count, uint32_t next_cap,
                        StrokeItem* pend, void* pend_pay, uint32_t* pend_count, uint32_t pend_cap,
                        uint32_t merge);

}  // namespace cvx

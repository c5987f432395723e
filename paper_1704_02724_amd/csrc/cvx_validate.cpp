// Host-side validation of node pools and views (no GPU calls).
//
// A pool is accepted when it is exactly the tree form of Sec. 4.1.1: roots
// [0, R^3), every refined cell owns one 8-aligned group of 8 consecutive
// children whose parent fields point back at it, no node is reached twice
// (no sharing, no cycles), depth never exceeds max_depth and every leaf index
// is in range with a finite, non-negative optical depth.  The breadth-first
// order produced here drives the level-by-level neighbour build on the GPU.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "cvx_internal.h"

namespace cvx {

static bool finite3(const double* v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

int check_desc(const cvx_canvas_desc* d, std::string& msg) {
  if (!d) { msg = "desc is NULL"; return CVX_ERR_INVALID_ARG; }
  if (d->R < 1 || d->R > 64) { msg = "R must be in [1, 64]"; return CVX_ERR_INVALID_ARG; }
  if (!(std::isfinite(d->root_edge) && d->root_edge > 0.0)) {
    msg = "root_edge must be finite and > 0";
    return CVX_ERR_INVALID_ARG;
  }
  if (!finite3(d->origin)) { msg = "origin must be finite"; return CVX_ERR_INVALID_ARG; }
  if (d->leaf_format != CVX_LEAF_RGBA8_F16 && d->leaf_format != CVX_LEAF_F64) {
    msg = "unknown leaf_format";
    return CVX_ERR_INVALID_ARG;
  }
  if (d->reserved != 0) { msg = "desc.reserved must be 0"; return CVX_ERR_INVALID_ARG; }
  if (d->max_depth > CVX_MAX_DEPTH) {
    msg = "max_depth exceeds CVX_MAX_DEPTH";
    return CVX_ERR_INVALID_ARG;
  }
  // cell coordinates at the deepest level, and the FP32 traversal's signed
  // plane offsets (at most R * 2^max_depth base cells), stay in int32 range
  if ((uint64_t)d->R << d->max_depth > (1ull << 30)) {
    msg = "R * 2^max_depth must not exceed 2^30";
    return CVX_ERR_INVALID_ARG;
  }
  return CVX_OK;
}

int validate_pool(const cvx_canvas_desc* desc, const cvx_node* nodes, uint64_t n_nodes,
                  const void* leaves, uint64_t n_leaves, PoolPlan* plan, std::string& msg) {
  int rc = check_desc(desc, msg);
  if (rc) return rc;
  const uint64_t R3 = (uint64_t)desc->R * desc->R * desc->R;
  const uint64_t P0 = (R3 + 7) & ~7ull;
  if (n_nodes < P0) { msg = "fewer nodes than the padded root array"; return CVX_ERR_BAD_POOL; }
  if (n_nodes > (uint64_t)CVX_LEAF_BIT) { msg = "more than 2^31 nodes"; return CVX_ERR_BAD_POOL; }
  if (!nodes) { msg = "nodes is NULL"; return CVX_ERR_INVALID_ARG; }
  if (n_leaves > (uint64_t)CVX_LEAF_BIT) { msg = "more than 2^31 leaves"; return CVX_ERR_BAD_POOL; }
  if (n_leaves && !leaves) { msg = "leaves is NULL"; return CVX_ERR_INVALID_ARG; }

  // leaf payload sanity
  if (desc->leaf_format == CVX_LEAF_RGBA8_F16) {
    const cvx_leaf_rgba8_f16* L = (const cvx_leaf_rgba8_f16*)leaves;
    for (uint64_t i = 0; i < n_leaves; ++i) {
      uint16_t h = L[i].kappa_f16;
      if ((h & 0x8000u) && (h & 0x7fffu)) { msg = "negative kappa in leaf " + std::to_string(i); return CVX_ERR_BAD_POOL; }
      if ((h & 0x7c00u) == 0x7c00u) { msg = "non-finite kappa in leaf " + std::to_string(i); return CVX_ERR_BAD_POOL; }
    }
  } else {
    const cvx_leaf_f64* L = (const cvx_leaf_f64*)leaves;
    for (uint64_t i = 0; i < n_leaves; ++i) {
      if (!(std::isfinite(L[i].kappa) && L[i].kappa >= 0.0) || !std::isfinite(L[i].r) ||
          !std::isfinite(L[i].g) || !std::isfinite(L[i].b)) {
        msg = "non-finite colour or negative/non-finite kappa in leaf " + std::to_string(i);
        return CVX_ERR_BAD_POOL;
      }
    }
  }

  std::vector<uint8_t> seen((n_nodes + 7) / 8, 0);
  auto test_and_set = [&](uint64_t i) {
    uint8_t m = (uint8_t)(1u << (i & 7));
    bool was = seen[i >> 3] & m;
    seen[i >> 3] |= m;
    return was;
  };
  std::vector<uint32_t> local;
  std::vector<uint32_t>& order = plan ? plan->order : local;
  order.clear();
  order.reserve(n_nodes);
  std::vector<uint64_t> level_off;
  level_off.push_back(0);
  for (uint64_t r = 0; r < R3; ++r) {
    if (nodes[r].parent != CVX_NONE) {
      msg = "root " + std::to_string(r) + " has a parent";
      return CVX_ERR_BAD_POOL;
    }
    test_and_set(r);
    order.push_back((uint32_t)r);
  }
  level_off.push_back(order.size());
  uint32_t depth = 0;
  for (;;) {
    uint64_t b = level_off[depth], e = level_off[depth + 1];
    if (b == e) break;
    for (uint64_t q = b; q < e; ++q) {
      uint32_t I = order[q];
      uint32_t c = nodes[I].child;
      if (c & CVX_LEAF_BIT) {
        if ((uint64_t)(c & ~CVX_LEAF_BIT) >= n_leaves) {
          msg = "node " + std::to_string(I) + ": leaf index out of range";
          return CVX_ERR_BAD_POOL;
        }
        continue;
      }
      if (c % 8 != 0) { msg = "node " + std::to_string(I) + ": child group not 8-aligned"; return CVX_ERR_BAD_POOL; }
      if ((uint64_t)c < P0 || (uint64_t)c + 8 > n_nodes) {
        msg = "node " + std::to_string(I) + ": child group out of range";
        return CVX_ERR_BAD_POOL;
      }
      if (depth + 1 > desc->max_depth) {
        msg = "node " + std::to_string(I) + ": depth exceeds max_depth";
        return CVX_ERR_BAD_POOL;
      }
      for (uint32_t o = 0; o < 8; ++o) {
        uint32_t ch = c + o;
        if (test_and_set(ch)) {
          msg = "node " + std::to_string(ch) + " is reached twice (shared group or cycle)";
          return CVX_ERR_BAD_POOL;
        }
        if (nodes[ch].parent != I) {
          msg = "node " + std::to_string(ch) + ": parent field does not match";
          return CVX_ERR_BAD_POOL;
        }
        order.push_back(ch);
      }
    }
    level_off.push_back(order.size());
    ++depth;
  }
  // depth = number of non-empty levels; deepest level index = depth - 1
  if (plan) {
    plan->level_off = level_off;
    plan->depth = depth ? depth - 1 : 0;
  }
  return CVX_OK;
}

int validate_views(const cvx_view* views, int n_views, const cvx_canvas_desc* const* canvases,
                   int n_canvases, std::string& msg) {
  if (!views || n_views < 1 || n_views > CVX_MAX_VIEWS) {
    msg = "n_views must be in [1, CVX_MAX_VIEWS] and views non-NULL";
    return CVX_ERR_INVALID_ARG;
  }
  for (int i = 0; i < n_views; ++i) {
    const cvx_view& v = views[i];
    std::string p = "view " + std::to_string(i) + ": ";
    if (v.canvas_id < 0 || v.canvas_id >= n_canvases || !canvases[v.canvas_id]) {
      msg = p + "canvas_id has no pool";
      return CVX_ERR_INVALID_ARG;
    }
    if (v.W < 1 || v.H < 1 || v.W > 65536 || v.H > 65536) {
      msg = p + "W and H must be in [1, 65536]";
      return CVX_ERR_INVALID_ARG;
    }
    if (!(v.alpha_stop > 0.0f)) { msg = p + "alpha_stop must be > 0"; return CVX_ERR_INVALID_ARG; }
    if (!finite3(v.eye) || !finite3(v.right) || !finite3(v.up) || !finite3(v.fwd)) {
      msg = p + "non-finite eye or basis";
      return CVX_ERR_INVALID_ARG;
    }
    if (!(std::isfinite(v.tan_half_fov_x) && v.tan_half_fov_x > 0 &&
          std::isfinite(v.tan_half_fov_y) && v.tan_half_fov_y > 0)) {
      msg = p + "tan_half_fov must be finite and > 0";
      return CVX_ERR_INVALID_ARG;
    }
    const double* b[3] = {v.right, v.up, v.fwd};
    for (int a = 0; a < 3; ++a) {
      for (int c = a; c < 3; ++c) {
        double dot = b[a][0] * b[c][0] + b[a][1] * b[c][1] + b[a][2] * b[c][2];
        double want = a == c ? 1.0 : 0.0;
        if (!(std::fabs(dot - want) < 1e-9)) {
          msg = p + "right/up/fwd must be orthonormal";
          return CVX_ERR_INVALID_ARG;
        }
      }
    }
    if (v.out_offset_px > (1ull << 48)) { msg = p + "out_offset_px too large"; return CVX_ERR_INVALID_ARG; }
  }
  return CVX_OK;
}

}  // namespace cvx

// Seeded-stroke canvas builder: turns a list of spherical brush stamps into
// the pointer-free octree node pool that the ray caster consumes.
//
// This is input generation only.  It implements the painting side of the
// method as a plain host program: spherical stamps (Sec. 5.1), the additive
// density/colour mix of Sec. 5.1 read with density as the alpha term, and the
// adaptive brush resolution of Sec. 5.2 (refine a cell that a stamp overlaps
// until its edge is at most radius/k, never past the maximum depth).  Trees
// always refine into 8 consecutive children (Sec. 4.1.1).  It contains no ray
// traversal and no compositing.
//
// Parallel build.  The tree above a split depth S is built sequentially; every
// depth-S cell X is then an independent subtree: the state of X when it is
// created (payload inherited from its parent, creating stroke s0) plus the
// ordered list of strokes s >= s0 that overlap X fully determine its subtree.
// Subtrees are built in parallel and the result is identical to a sequential
// build for every thread count.
//
// Output (emitted in depth-first group order for locality):
//   nodes  : uint32 pairs {child, parent}; child has bit 31 set for a leaf and
//            then indexes the leaf array, otherwise it is the first of 8
//            consecutive children.  Roots are nodes [0, R^3) x-fastest, padded
//            to a multiple of 8; padding slots are leaves of the first root's
//            payload with parent 0xffffffff and are never referenced.
//   leaves : format 0 -> {u8 r,g,b,a; u16 kappa_f16; u16 pad}
//            format 1 -> {double r,g,b,kappa}
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr uint32_t LEAF = 0x80000000u;
constexpr uint32_t NONE = 0xffffffffu;

struct Stamp { double x, y, z, r; };

struct Strokes {
  int n;
  const int64_t* off;      // n+1 offsets into stamps
  const Stamp* stamps;
  const double* rgb;       // 3 per stroke
  const double* sigma;     // per stroke
  const double* radius;    // per stroke
};

// Squared distance from a point to a closed axis-aligned box.
inline double box_dist2(double lx, double ly, double lz, double e, const Stamp& s) {
  double d2 = 0.0, v;
  v = std::max(std::max(lx - s.x, 0.0), s.x - (lx + e)); d2 += v * v;
  v = std::max(std::max(ly - s.y, 0.0), s.y - (ly + e)); d2 += v * v;
  v = std::max(std::max(lz - s.z, 0.0), s.z - (lz + e)); d2 += v * v;
  return d2;
}

template <class T>
struct Pool {
  std::vector<uint32_t> child;   // LEAF or first child
  std::vector<uint32_t> mark;    // last stroke (+1) that painted the cell
  std::vector<T> col;            // r,g,b,kappa per node
  std::vector<int32_t> ext;      // for the top tree: index of the depth-S subtree, else -1

  uint32_t size() const { return (uint32_t)child.size(); }
  uint32_t add_group(const T* inherit) {
    uint32_t g = size();
    for (int o = 0; o < 8; ++o) {
      child.push_back(LEAF);
      mark.push_back(0);
      for (int c = 0; c < 3; ++c) col.push_back(inherit[c]);
      col.push_back(inherit[3] * T(0.5));  // optical depth per leaf edge halves
      ext.push_back(-1);
    }
    return g;
  }
};

struct SubtreeSeed {
  int ix, iy, iz;      // coordinates at depth S
  int s0;              // creating stroke
  double col[4];       // inherited payload at creation
};

template <class T>
struct Builder {
  uint32_t R, D, S;
  double k, root_edge;
  Strokes st;
  struct Item { uint32_t node; int d; int64_t x, y, z; };

  // paint-or-refine one stamp into the subtree rooted at `root` (a cell of
  // depth d0 with integer coords (x0,y0,z0)); cells at depth `stop` are not
  // entered (they are recorded through `on_stop`).
  template <class OnStop>
  void apply_stamp(Pool<T>& P, uint32_t root, int d0, int64_t x0, int64_t y0, int64_t z0,
                   int stroke, const Stamp& sp, uint32_t stop, OnStop&& on_stop) {
    Item stack[8 * 40];
    int top = 0;
    stack[top++] = {root, d0, x0, y0, z0};
    const double rr = sp.r * sp.r;
    const double hmin = st.radius[stroke] / k;
    while (top) {
      Item it = stack[--top];
      double e = std::ldexp(root_edge, -it.d);
      double lx = it.x * e, ly = it.y * e, lz = it.z * e;
      if (!(box_dist2(lx, ly, lz, e, sp) < rr)) continue;
      if ((uint32_t)it.d == stop) { on_stop(it.node); continue; }
      uint32_t c = P.child[it.node];
      if (c & LEAF) {
        if (e > hmin && (uint32_t)it.d < D) {
          T inh[4] = {P.col[4 * it.node], P.col[4 * it.node + 1], P.col[4 * it.node + 2],
                      P.col[4 * it.node + 3]};
          c = P.add_group(inh);
          P.child[it.node] = c;
          if ((uint32_t)(it.d + 1) == stop) {
            for (int o = 0; o < 8; ++o) on_create(P, c + o, it, o, stroke);
          }
        } else {
          double cx = lx + 0.5 * e - sp.x, cy = ly + 0.5 * e - sp.y, cz = lz + 0.5 * e - sp.z;
          if (cx * cx + cy * cy + cz * cz <= rr && P.mark[it.node] != (uint32_t)stroke + 1) {
            P.mark[it.node] = (uint32_t)stroke + 1;
            T* q = &P.col[4 * it.node];
            double kb = st.sigma[stroke] * e / st.radius[stroke];
            double kc = (double)q[3];
            double m = kb / (kb + kc);
            for (int ch = 0; ch < 3; ++ch)
              q[ch] = (T)(m * st.rgb[3 * stroke + ch] + (1.0 - m) * (double)q[ch]);
            q[3] = (T)(kb + kc);
          }
          continue;
        }
      }
      for (int o = 7; o >= 0; --o)
        stack[top++] = {c + (uint32_t)o, it.d + 1, 2 * it.x + (o & 1), 2 * it.y + ((o >> 1) & 1),
                        2 * it.z + ((o >> 2) & 1)};
    }
  }

  std::vector<SubtreeSeed> seeds;
  void on_create(Pool<T>& P, uint32_t node, const Item& par, int o, int stroke) {
    const Item* it = &par;
    SubtreeSeed sd;
    sd.ix = (int)(2 * it->x + (o & 1));
    sd.iy = (int)(2 * it->y + ((o >> 1) & 1));
    sd.iz = (int)(2 * it->z + ((o >> 2) & 1));
    sd.s0 = stroke;
    for (int c = 0; c < 4; ++c) sd.col[c] = (double)P.col[4 * node + c];
    P.ext[node] = (int32_t)seeds.size();
    seeds.push_back(sd);
  }
};

// Result handle handed back to the caller.
struct Result {
  std::vector<uint32_t> nodes;   // 2 per node
  std::vector<uint8_t> leaves;   // packed leaf records
  uint64_t n_nodes = 0, n_leaves = 0;
  uint32_t max_depth_seen = 0;
  std::vector<uint64_t> depth_hist;  // leaves per depth
};

uint16_t f32_to_f16(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  uint32_t sign = (x >> 16) & 0x8000u;
  uint32_t ex = (x >> 23) & 0xffu, man = x & 0x7fffffu;
  if (ex == 0xffu) return (uint16_t)(sign | 0x7c00u | (man ? 0x200u : 0u));
  int e = (int)ex - 127 + 15;
  if (e >= 31) return (uint16_t)(sign | 0x7c00u);
  if (e <= 0) {
    if (e < -10) return (uint16_t)sign;
    man |= 0x800000u;
    int shift = 14 - e;
    uint32_t h = man >> shift, rem = man & ((1u << shift) - 1u), half = 1u << (shift - 1);
    if (rem > half || (rem == half && (h & 1u))) ++h;
    return (uint16_t)(sign | h);
  }
  uint32_t h = sign | ((uint32_t)e << 10) | (man >> 13);
  uint32_t rem = man & 0x1fffu;
  if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;
  return (uint16_t)h;
}

template <class T>
void emit_leaf(Result& res, uint64_t li, const T* c, int fmt) {
  if (fmt == 0) {
    uint8_t* p = &res.leaves[li * 8];
    for (int ch = 0; ch < 3; ++ch) {
      double v = std::min(std::max((double)c[ch], 0.0), 1.0);
      p[ch] = (uint8_t)std::lrint(255.0 * v);
    }
    double kap = std::max((double)c[3], 0.0);
    p[3] = (uint8_t)std::lrint(255.0 * (1.0 - std::exp(-kap)));
    uint16_t h = f32_to_f16((float)std::min(kap, 65504.0));
    std::memcpy(p + 4, &h, 2);
    p[6] = p[7] = 0;
  } else {
    double v[4] = {(double)c[0], (double)c[1], (double)c[2], (double)c[3]};
    std::memcpy(&res.leaves[li * 32], v, 32);
  }
}

// Progress lines on stderr for long builds (set by cg_set_verbose).
std::atomic<int> g_verbose{0};

template <class T>
int build(uint32_t R, uint32_t D, double k, uint32_t S, int nthreads, const Strokes& st, int fmt,
          Result& res) {
  Builder<T> B;
  B.R = R; B.D = D; B.k = k; B.st = st;
  B.root_edge = 1.0 / (double)R;
  B.S = (S == 0 || S > D) ? D + 1 : S;  // no split when S is past the max depth
  const uint32_t R3 = R * R * R;
  const uint32_t P0 = (R3 + 7u) & ~7u;

  Pool<T> top;
  top.child.assign(P0, LEAF);
  top.mark.assign(P0, 0);
  top.col.assign(4 * (size_t)P0, T(0));
  top.ext.assign(P0, -1);

  auto root_range = [&](const Stamp& sp, int axis, int& lo, int& hi) {
    double c = axis == 0 ? sp.x : axis == 1 ? sp.y : sp.z;
    lo = (int)std::floor((c - sp.r) * R);
    hi = (int)std::floor((c + sp.r) * R);
    lo = std::max(lo, 0);
    hi = std::min(hi, (int)R - 1);
  };

  // Phase 1: everything above depth S (or the whole tree when S > D).
  for (int s = 0; s < st.n; ++s) {
    for (int64_t j = st.off[s]; j < st.off[s + 1]; ++j) {
      const Stamp& sp = st.stamps[j];
      int xl, xh, yl, yh, zl, zh;
      root_range(sp, 0, xl, xh); root_range(sp, 1, yl, yh); root_range(sp, 2, zl, zh);
      for (int z = zl; z <= zh; ++z)
        for (int y = yl; y <= yh; ++y)
          for (int x = xl; x <= xh; ++x) {
            uint32_t root = (uint32_t)(x + (int)R * (y + (int)R * z));
            B.apply_stamp(top, root, 0, x, y, z, s, sp, B.S, [](uint32_t) {});
          }
    }
  }
  if (B.S == 0) return -1;  // unreachable: roots are never split points

  // Phase 2: independent subtrees rooted at depth S.
  const size_t nsub = B.seeds.size();
  std::vector<Pool<T>> subs(nsub);
  if (nsub) {
    // Stroke lists per subtree (strokes >= s0 whose stamps overlap X).
    std::vector<std::vector<int>> lists(nsub);
    const uint64_t side = (uint64_t)R << B.S;
    // dense map depth-S coords -> seed index (only cells that exist)
    std::vector<int32_t> grid;
    bool dense = side <= 512;
    if (dense) {
      grid.assign(side * side * side, -1);
      for (size_t i = 0; i < nsub; ++i) {
        const auto& sd = B.seeds[i];
        grid[((uint64_t)sd.iz * side + sd.iy) * side + sd.ix] = (int32_t)i;
      }
    }
    std::vector<int> lastmark(nsub, -1);
    double e = std::ldexp(B.root_edge, -(int)B.S);
    for (int s = 0; s < st.n; ++s) {
      for (int64_t j = st.off[s]; j < st.off[s + 1]; ++j) {
        const Stamp& sp = st.stamps[j];
        int64_t lo[3], hi[3];
        double c[3] = {sp.x, sp.y, sp.z};
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::max<int64_t>((int64_t)std::floor((c[a] - sp.r) / e), 0);
          hi[a] = std::min<int64_t>((int64_t)std::floor((c[a] + sp.r) / e), (int64_t)side - 1);
        }
        if (!dense) return -2;
        for (int64_t z = lo[2]; z <= hi[2]; ++z)
          for (int64_t y = lo[1]; y <= hi[1]; ++y)
            for (int64_t x = lo[0]; x <= hi[0]; ++x) {
              int32_t id = grid[((uint64_t)z * side + y) * side + x];
              if (id < 0 || lastmark[id] == s || B.seeds[id].s0 > s) continue;
              if (!(box_dist2(x * e, y * e, z * e, e, sp) < sp.r * sp.r)) continue;
              lastmark[id] = s;
              lists[id].push_back(s);
            }
      }
    }
    std::vector<size_t> order(nsub);
    for (size_t i = 0; i < nsub; ++i) order[i] = i;
    std::sort(order.begin(), order.end(),
              [&](size_t a, size_t b) { return lists[a].size() > lists[b].size(); });
    std::atomic<size_t> next{0}, done{0};
    if (g_verbose)
      std::fprintf(stderr, "[canvasgen] top tree built, painting %zu subtrees\n", nsub);
    auto work = [&]() {
      for (;;) {
        size_t w = next.fetch_add(1);
        if (w >= nsub) break;
        size_t i = order[w];
        const auto& sd = B.seeds[i];
        Pool<T>& P = subs[i];
        P.child.push_back(LEAF);
        P.mark.push_back(0);
        for (int c2 = 0; c2 < 4; ++c2) P.col.push_back((T)sd.col[c2]);
        P.ext.push_back(-1);
        for (int s : lists[i])
          for (int64_t j = st.off[s]; j < st.off[s + 1]; ++j)
            B.apply_stamp(P, 0, (int)B.S, sd.ix, sd.iy, sd.iz, s, st.stamps[j], 0xffffffffu,
                          [](uint32_t) {});
        const size_t d = done.fetch_add(1) + 1;
        if (g_verbose && nsub >= 10 && d % (nsub / 10) == 0)
          std::fprintf(stderr, "[canvasgen] painted %zu / %zu subtrees\n", d, nsub);
      }
    };
    int nt = std::max(1, nthreads);
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
  }

  if (g_verbose) std::fprintf(stderr, "[canvasgen] emitting the pool\n");
  // Emit in depth-first group order.  Count first.
  uint64_t nn = P0, nl = 0;
  {
    // top tree: every non-root node is in a group; subtree roots are top nodes
    uint64_t top_groups = (top.size() - P0) / 8;
    nn += top_groups * 8;
    for (auto& P : subs) nn += P.size() - 1;
  }
  if (nn >= (uint64_t)LEAF) return -3;
  res.n_nodes = nn;
  res.nodes.assign(2 * nn, 0);
  res.depth_hist.assign(64, 0);
  // leaf count
  for (uint32_t i = 0; i < top.size(); ++i)
    if ((top.child[i] & LEAF) && top.ext[i] < 0 && (i >= P0 || i < R3)) ++nl;
  for (auto& P : subs)
    for (uint32_t i = 0; i < P.size(); ++i)
      if (P.child[i] & LEAF) ++nl;
  res.n_leaves = nl;
  res.leaves.assign(nl * (fmt == 0 ? 8 : 32), 0);

  uint64_t next_node = P0, next_leaf = 0;
  struct Frame { const Pool<T>* P; uint32_t src; uint64_t dst; uint32_t parent_dst; int d; };
  std::vector<Frame> stack;
  auto emit = [&](const Pool<T>* P, uint32_t src, uint64_t dst, uint32_t parent_dst, int d) {
    stack.push_back({P, src, dst, parent_dst, d});
    while (!stack.empty()) {
      Frame f = stack.back();
      stack.pop_back();
      const Pool<T>* Q = f.P;
      uint32_t s2 = f.src;
      if (Q == &top && top.ext[s2] >= 0) {
        Q = &subs[top.ext[s2]];
        s2 = 0;
      }
      res.nodes[2 * f.dst + 1] = f.parent_dst;
      uint32_t c = Q->child[s2];
      if (c & LEAF) {
        res.nodes[2 * f.dst] = LEAF | (uint32_t)next_leaf;
        emit_leaf<T>(res, next_leaf, &Q->col[4 * (size_t)s2], fmt);
        ++next_leaf;
        res.depth_hist[f.d]++;
        res.max_depth_seen = std::max(res.max_depth_seen, (uint32_t)f.d);
      } else {
        uint64_t g = next_node;
        next_node += 8;
        res.nodes[2 * f.dst] = (uint32_t)g;
        for (int o = 7; o >= 0; --o)
          stack.push_back({Q, c + (uint32_t)o, g + (uint64_t)o, (uint32_t)f.dst, f.d + 1});
      }
    }
  };
  for (uint32_t r = 0; r < R3; ++r) emit(&top, r, r, NONE, 0);
  // padding root slots: leaves sharing leaf 0, never referenced
  for (uint32_t r = R3; r < P0; ++r) {
    res.nodes[2 * r] = LEAF | 0u;
    res.nodes[2 * r + 1] = NONE;
  }
  if (next_node != nn || next_leaf != nl) return -4;
  return 0;
}

}  // namespace

extern "C" {

// Builds a canvas.  Returns 0 and an opaque handle on success, < 0 on error.
int cg_build(uint32_t R, uint32_t max_depth, double k_refine, uint32_t split_depth, int nthreads,
             int n_strokes, const int64_t* stamp_off, const double* stamps, const double* rgb,
             const double* sigma, const double* radius, int leaf_format, void** handle) {
  if (!handle || R == 0 || R > 64 || max_depth > 31 || !(k_refine > 0) || n_strokes < 0 ||
      (leaf_format != 0 && leaf_format != 1))
    return -10;
  Strokes st{n_strokes, stamp_off, (const Stamp*)stamps, rgb, sigma, radius};
  Result* res = new (std::nothrow) Result();
  if (!res) return -11;
  int rc;
  try {
    if (leaf_format == 1)
      rc = build<double>(R, max_depth, k_refine, split_depth, nthreads, st, leaf_format, *res);
    else
      rc = build<float>(R, max_depth, k_refine, split_depth, nthreads, st, leaf_format, *res);
  } catch (const std::bad_alloc&) {
    rc = -12;
  }
  if (rc != 0) {
    delete res;
    return rc;
  }
  *handle = res;
  return 0;
}

void cg_result_sizes(void* h, uint64_t* n_nodes, uint64_t* n_leaves, uint32_t* max_depth_seen) {
  Result* r = (Result*)h;
  *n_nodes = r->n_nodes;
  *n_leaves = r->n_leaves;
  *max_depth_seen = r->max_depth_seen;
}

void cg_result_copy(void* h, uint32_t* nodes, void* leaves, uint64_t* depth_hist64) {
  Result* r = (Result*)h;
  if (nodes) std::memcpy(nodes, r->nodes.data(), r->nodes.size() * 4);
  if (leaves) std::memcpy(leaves, r->leaves.data(), r->leaves.size());
  if (depth_hist64) std::memcpy(depth_hist64, r->depth_hist.data(), 64 * 8);
}

void cg_result_free(void* h) { delete (Result*)h; }

// Nonzero: long builds print progress lines on stderr.
void cg_set_verbose(int v) { g_verbose = v; }

uint16_t cg_f32_to_f16(float f) { return f32_to_f16(f); }

}  // extern "C"

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

// The painted trees of one build, kept until they are emitted: the tree
// above the split depth and one pool per depth-S subtree.
template <class T>
struct Painted {
  uint32_t R = 1, P0 = 8;
  Pool<T> top;
  std::vector<Pool<T>> subs;
  std::vector<uint64_t> sub_leaves;  // leaves per subtree
};

// Result handle handed back to the caller: sizes after the build, the pool
// itself after emission into the caller's arrays.
struct Result {
  uint64_t n_nodes = 0, n_leaves = 0;
  int fmt = 0;
  Painted<float>* pf = nullptr;
  Painted<double>* pd = nullptr;
  ~Result() {
    delete pf;
    delete pd;
  }
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
void emit_leaf(uint8_t* leaves, uint64_t li, const T* c, int fmt) {
  if (fmt == 0) {
    uint8_t* p = &leaves[li * 8];
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
    std::memcpy(&leaves[li * 32], v, 32);
  }
}

// Progress lines on stderr for long builds (set by cg_set_verbose).
std::atomic<int> g_verbose{0};

template <class T>
int build(uint32_t R, uint32_t D, double k, uint32_t S, int nthreads, const Strokes& st,
          Painted<T>& out, uint64_t& n_nodes, uint64_t& n_leaves) {
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
  std::vector<Pool<T>>& subs = out.subs;
  subs.assign(nsub, Pool<T>());
  out.sub_leaves.assign(nsub, 0);
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
        uint64_t nl = 0;
        for (uint32_t c : P.child) nl += (c & LEAF) ? 1u : 0u;
        out.sub_leaves[i] = nl;
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

  // sizes of the pool in depth-first group order
  uint64_t nn = P0, nl = 0;
  {
    // top tree: every non-root node is in a group; subtree roots are top nodes
    uint64_t top_groups = (top.size() - P0) / 8;
    nn += top_groups * 8;
    for (auto& P : subs) nn += P.size() - 1;
  }
  if (nn >= (uint64_t)LEAF) return -3;
  for (uint32_t i = 0; i < top.size(); ++i)
    if ((top.child[i] & LEAF) && top.ext[i] < 0 && (i >= P0 || i < R3)) ++nl;
  for (uint64_t c : out.sub_leaves) nl += c;
  out.R = R;
  out.P0 = P0;
  out.top = std::move(top);
  n_nodes = nn;
  n_leaves = nl;
  return 0;
}

// Depth-first emission of one tree below `src` of pool P (dst: its output
// node id), allocating groups from next_node and leaves from next_leaf in
// the order a preorder walk meets them.  A top-tree node standing for a
// depth-S subtree is emitted from that subtree's pool unless `stop_at_subs`
// asks for it to be handed to on_sub instead (which then reserves the
// subtree's contiguous node and leaf ranges).
template <class T, class OnSub>
void emit_tree(const Painted<T>& W, const Pool<T>* P, uint32_t src, uint64_t dst,
               uint32_t parent_dst, int d, uint32_t* nodes, uint8_t* leaves, int fmt,
               uint64_t& next_node, uint64_t& next_leaf, uint64_t* hist, uint32_t& md,
               bool stop_at_subs, OnSub&& on_sub) {
  struct Frame { const Pool<T>* P; uint32_t src; uint64_t dst; uint32_t parent_dst; int d; };
  std::vector<Frame> stack;
  stack.push_back({P, src, dst, parent_dst, d});
  while (!stack.empty()) {
    Frame f = stack.back();
    stack.pop_back();
    const Pool<T>* Q = f.P;
    uint32_t s2 = f.src;
    nodes[2 * f.dst + 1] = f.parent_dst;
    if (Q == &W.top && W.top.ext[s2] >= 0) {
      const int32_t e = W.top.ext[s2];
      if (stop_at_subs) {
        on_sub(e, f.dst, f.d);
        continue;
      }
      Q = &W.subs[e];
      s2 = 0;
    }
    uint32_t c = Q->child[s2];
    if (c & LEAF) {
      nodes[2 * f.dst] = LEAF | (uint32_t)next_leaf;
      emit_leaf<T>(leaves, next_leaf, &Q->col[4 * (size_t)s2], fmt);
      ++next_leaf;
      hist[f.d]++;
      md = std::max(md, (uint32_t)f.d);
    } else {
      uint64_t g = next_node;
      next_node += 8;
      nodes[2 * f.dst] = (uint32_t)g;
      for (int o = 7; o >= 0; --o)
        stack.push_back({Q, c + (uint32_t)o, g + (uint64_t)o, (uint32_t)f.dst, f.d + 1});
    }
  }
}

// Emission into the caller's arrays.  A preorder walk allocates the groups
// of a subtree's descendants contiguously (the walk finishes a subtree before
// it pops anything pushed earlier), so the walk of the top tree reserves each
// depth-S subtree's node and leaf ranges and the subtrees are emitted in
// parallel into them: the output is the sequential walk's, byte for byte.
template <class T>
int emit(const Painted<T>& W, uint64_t nn, uint64_t nl, uint32_t* nodes, uint8_t* leaves, int fmt,
         uint64_t* hist_out, uint32_t* md_out, int nthreads) {
  if (g_verbose) std::fprintf(stderr, "[canvasgen] emitting the pool\n");
  struct Task { int32_t sub; uint64_t dst, node_base, leaf_base; int d; };
  std::vector<Task> tasks;
  uint64_t next_node = W.P0, next_leaf = 0;
  std::vector<uint64_t> hist(64, 0);
  uint32_t md = 0;
  const uint32_t R3 = W.R * W.R * W.R;
  for (uint32_t r = 0; r < R3; ++r)
    emit_tree<T>(W, &W.top, r, r, NONE, 0, nodes, leaves, fmt, next_node, next_leaf, hist.data(),
                 md, true, [&](int32_t e, uint64_t dst, int d) {
                   const Pool<T>& P = W.subs[e];
                   if (P.child[0] & LEAF) {  // an unrefined subtree root: one leaf
                     nodes[2 * dst] = LEAF | (uint32_t)next_leaf;
                     emit_leaf<T>(leaves, next_leaf, &P.col[0], fmt);
                     ++next_leaf;
                     hist[d]++;
                     md = std::max(md, (uint32_t)d);
                     return;
                   }
                   tasks.push_back({e, dst, next_node, next_leaf, d});
                   next_node += P.size() - 1;
                   next_leaf += W.sub_leaves[e];
                 });
  // padding root slots: leaves sharing leaf 0, never referenced
  for (uint32_t r = R3; r < W.P0; ++r) {
    nodes[2 * r] = LEAF | 0u;
    nodes[2 * r + 1] = NONE;
  }
  if (next_node != nn || next_leaf != nl) return -4;
  std::atomic<size_t> next{0};
  std::vector<std::vector<uint64_t>> hists(std::max(1, nthreads), std::vector<uint64_t>(64, 0));
  std::vector<uint32_t> mds(std::max(1, nthreads), 0);
  std::atomic<int> bad{0};
  auto work = [&](int t) {
    for (;;) {
      const size_t i = next.fetch_add(1);
      if (i >= tasks.size()) break;
      const Task& k = tasks[i];
      const Pool<T>& P = W.subs[k.sub];
      uint64_t nn_t = k.node_base, nl_t = k.leaf_base;
      // the subtree root's own record: its group is the first of its range
      nodes[2 * k.dst] = (uint32_t)nn_t;
      const uint32_t c = P.child[0];
      nn_t += 8;
      for (uint32_t o = 0; o < 8; ++o)
        emit_tree<T>(W, &P, c + o, k.node_base + o, (uint32_t)k.dst, k.d + 1, nodes, leaves, fmt,
                     nn_t, nl_t, hists[t].data(), mds[t], false, [](int32_t, uint64_t, int) {});
      if (nn_t != k.node_base + P.size() - 1 || nl_t != k.leaf_base + W.sub_leaves[k.sub])
        bad = 1;
    }
  };
  int nt = std::max(1, nthreads);
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& t : th) t.join();
  if (bad) return -4;
  for (int t = 0; t < nt; ++t) {
    for (int j = 0; j < 64; ++j) hist[j] += hists[t][j];
    md = std::max(md, mds[t]);
  }
  if (hist_out) std::memcpy(hist_out, hist.data(), 64 * 8);
  if (md_out) *md_out = md;
  return 0;
}

}  // namespace

extern "C" {

// Builds a canvas (paints every stroke into the trees).  Returns 0 and an
// opaque handle on success, < 0 on error; cg_result_sizes then gives the
// pool's size and cg_emit writes it.
int cg_build(uint32_t R, uint32_t max_depth, double k_refine, uint32_t split_depth, int nthreads,
             int n_strokes, const int64_t* stamp_off, const double* stamps, const double* rgb,
             const double* sigma, const double* radius, int leaf_format, void** handle) {
  if (!handle || R == 0 || R > 64 || max_depth > 31 || !(k_refine > 0) || n_strokes < 0 ||
      (leaf_format != 0 && leaf_format != 1))
    return -10;
  Strokes st{n_strokes, stamp_off, (const Stamp*)stamps, rgb, sigma, radius};
  Result* res = new (std::nothrow) Result();
  if (!res) return -11;
  res->fmt = leaf_format;
  int rc;
  try {
    if (leaf_format == 1) {
      res->pd = new Painted<double>();
      rc = build<double>(R, max_depth, k_refine, split_depth, nthreads, st, *res->pd,
                         res->n_nodes, res->n_leaves);
    } else {
      res->pf = new Painted<float>();
      rc = build<float>(R, max_depth, k_refine, split_depth, nthreads, st, *res->pf,
                        res->n_nodes, res->n_leaves);
    }
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

void cg_result_sizes(void* h, uint64_t* n_nodes, uint64_t* n_leaves) {
  Result* r = (Result*)h;
  *n_nodes = r->n_nodes;
  *n_leaves = r->n_leaves;
}

// Writes the pool into the caller's arrays: nodes (2 uint32 per node), leaves
// (8 or 32 bytes per leaf), leaves per depth (64 uint64) and the deepest
// leaf depth.  Returns 0, or < 0 if the emission disagrees with the sizes.
int cg_emit(void* h, uint32_t* nodes, void* leaves, uint64_t* depth_hist64,
            uint32_t* max_depth_seen, int nthreads) {
  Result* r = (Result*)h;
  try {
    if (r->pd)
      return emit<double>(*r->pd, r->n_nodes, r->n_leaves, nodes, (uint8_t*)leaves, r->fmt,
                          depth_hist64, max_depth_seen, nthreads);
    return emit<float>(*r->pf, r->n_nodes, r->n_leaves, nodes, (uint8_t*)leaves, r->fmt,
                       depth_hist64, max_depth_seen, nthreads);
  } catch (const std::bad_alloc&) {
    return -12;
  }
}

void cg_result_free(void* h) { delete (Result*)h; }

// Nonzero: long builds print progress lines on stderr.
void cg_set_verbose(int v) { g_verbose = v; }

uint16_t cg_f32_to_f16(float f) { return f32_to_f16(f); }

}  // extern "C"

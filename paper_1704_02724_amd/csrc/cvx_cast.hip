// Ray-casting kernels for deep-octree canvases (CDNA4 / gfx950).
//
// One lane traces one pixel's ray; a persistent grid of wavefronts pulls
// 64-pixel tiles (or 64-ray chunks in trace mode) from a device work queue.
// Every pixel is computed by exactly one lane with a fixed per-ray operation
// order, so results do not depend on scheduling.
//
// Traversal (Sec. 6.2): from the entry point of the current leaf, find the
// exit face and the traversal length, step to the neighbour across that face
// - a sibling by index arithmetic, or the stored outer-face link (G_3) - and,
// when the neighbour is refined, descend to the child that contains the exit
// point (Sec. 4.1.1, first child + octant).  Colour accumulates front to back
// until the ray leaves the canvas or reaches the stop opacity.
//
// Three variants share the integer bookkeeping (node id, depth, integer cell
// coordinates at that depth, which makes every face plane an exact dyadic):
//  FP32_REBASED  cell-local FP32 point p in [-0.5,0.5]^3 (Sec. 6.1-6.3: origin
//                at the cell centre, edge 1).  Exit lengths t_k =
//                (+-0.5 - p_k)/d_k in FP32 with a running error bound on p in
//                the spirit of the per-step analysis of Sec. 6.3; an exit
//                decision whose margin is below the bound is re-taken in FP64
//                from the exact face planes.  On every descent, after such a
//                fallback, or once the bound has grown, p is rebuilt from the
//                FP64 ray at the exactly known crossing plane ("rebase").
//                Same-depth steps only flip p on the exit axis; steps into a
//                coarser leaf rescale p by a power of two.
//  FP64_PLAIN    canvas-global FP64: exit t from the exact face planes, FP64
//                compositing.  The GPU baseline.
//  FP32_NAIVE    canvas-global FP32 (the paper's "canvas coordinate"
//                traversal that drifts at depth); kept to show the failure.
#include <hip/hip_runtime.h>

#include "cvx_internal.h"

namespace cvx {

namespace {

constexpr float BIGF = 1e30f;
constexpr float EP_MAX = 0x1p-14f;  // rebase once the point error bound exceeds this

struct Acc {
  uint32_t rays, leaves, outer, descent, fp64_exit, rebase;
};

// Runtime-indexed access to 3-element register arrays without private memory.
template <class T>
__device__ __forceinline__ T pick(const T a[3], int k) {
  return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]);
}
template <class T>
__device__ __forceinline__ void put(T a[3], int k, T v) {
  a[0] = k == 0 ? v : a[0];
  a[1] = k == 1 ? v : a[1];
  a[2] = k == 2 ? v : a[2];
}

__device__ __forceinline__ void ray_dir(const DView& v, uint32_t x, uint32_t y, double d[3]) {
#pragma clang fp contract(off)
  double u = (2.0 * ((double)x + 0.5) / (double)v.W - 1.0) * v.tan_x;
  double w = (1.0 - 2.0 * ((double)y + 0.5) / (double)v.H) * v.tan_y;
  double n2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    d[k] = v.fwd[k] + u * v.right[k];
    d[k] = d[k] + w * v.up[k];
    n2 += d[k] * d[k];
  }
  double n = __builtin_sqrt(n2);
  for (int k = 0; k < 3; ++k) d[k] = d[k] / n;
}

struct Entry {
  double t0, t1;
  int kin, side;
  bool hit;
};

// Slab test of the ray against the canvas box [0, R]^3 (FP64).
__device__ __forceinline__ Entry canvas_entry(const double o[3], const double d[3], double Rd) {
  Entry e;
  double tin = -__builtin_inf(), tout = __builtin_inf();
  int kin = -1, side = 0;
  bool miss = false;
  for (int k = 0; k < 3; ++k) {
    if (d[k] != 0.0) {
      double ta = (0.0 - o[k]) / d[k], tb = (Rd - o[k]) / d[k];
      double lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
      if (lo > tin) {
        tin = lo;
        kin = k;
        side = d[k] > 0.0 ? 0 : 1;
      }
      if (hi < tout) tout = hi;
    } else if (o[k] < 0.0 || o[k] > Rd) {
      miss = true;
    }
  }
  e.t0 = tin > 0.0 ? tin : 0.0;
  e.t1 = tout;
  e.kin = tin > 0.0 ? kin : -1;
  e.side = side;
  e.hit = !miss && e.t0 < e.t1;
  return e;
}

__device__ __forceinline__ uint4 ld_rec(const void* rec, uint32_t i) {
  return ((const uint4*)rec)[i];
}

// Descend from the current cell (r refined) to the leaf containing q; on a
// mid-plane the child on the side the ray moves into is taken.
template <class Real>
__device__ __forceinline__ void descend(const void* rec, const Real q[3], const bool up[3],
                                        uint32_t& I, uint32_t& dep, uint32_t c[3], uint4& r) {
  while (!(r.x & 1u)) {
    Real h = (Real)ldexp(1.0, -(int)dep);
    uint32_t oct = 0;
    for (int k = 0; k < 3; ++k) {
      Real mid = ((Real)c[k] + (Real)0.5) * h;
      uint32_t b = (q[k] > mid) || (q[k] == mid && up[k]);
      oct |= b << k;
      c[k] = 2u * c[k] + b;
    }
    I = r.x + oct;
    ++dep;
    r = ld_rec(rec, I);
  }
}

// Root cell containing q (ties go to the side the ray moves into).
template <class Real>
__device__ __forceinline__ void root_of(const Real q[3], const bool up[3], uint32_t R,
                                        uint32_t c[3], uint32_t& I) {
  for (int k = 0; k < 3; ++k) {
    Real f = floor(q[k]);
    int n = (int)f;
    if (q[k] == f && !up[k]) n -= 1;
    n = n < 0 ? 0 : n;
    n = n > (int)R - 1 ? (int)R - 1 : n;
    c[k] = (uint32_t)n;
  }
  I = c[0] + R * (c[1] + R * c[2]);
}

__device__ __forceinline__ void decode8(uint2 p, float col[3], float& kap) {
  col[0] = (float)(p.x & 0xffu) * (1.0f / 255.0f);
  col[1] = (float)((p.x >> 8) & 0xffu) * (1.0f / 255.0f);
  col[2] = (float)((p.x >> 16) & 0xffu) * (1.0f / 255.0f);
  kap = (float)__builtin_bit_cast(_Float16, (unsigned short)(p.y & 0xffffu));
}

struct Out {
  double rgba[4];
  uint32_t flags;
  uint32_t n;
};

// Trace sink: records (leaf, l) pairs when tracing is on.
struct Sink {
  uint32_t* ids;
  float* len32;
  double* len64;
  uint32_t cap;
};

template <int VAR, bool TRACE, bool STATS>
__device__ void cast_ray(const DView& v, uint32_t px, uint32_t py, Sink sk, Acc& acc, Out& out) {
  double d[3];
  ray_dir(v, px, py, d);
  const double o[3] = {v.o[0], v.o[1], v.o[2]};
  const double Rd = (double)v.R;
  const void* rec = v.rec;
  out.rgba[0] = out.rgba[1] = out.rgba[2] = out.rgba[3] = 0.0;
  out.flags = 0;
  out.n = 0;
  if (STATS) acc.rays++;
  Entry en = canvas_entry(o, d, Rd);
  if (!en.hit) return;
  const bool up[3] = {d[0] > 0.0, d[1] > 0.0, d[2] > 0.0};
  const bool use_stop = v.alpha_stop < 1.0f;
  uint32_t n_rec = 0;

  // ---------------------------------------------------------------- FP32 naive
  if constexpr (VAR == (int)CVX_VARIANT_FP32_NAIVE) {
    float of[3], df[3], idf[3];
    bool par[3];
    for (int k = 0; k < 3; ++k) {
      of[k] = (float)o[k];
      df[k] = (float)d[k];
      par[k] = df[k] == 0.0f;
      idf[k] = par[k] ? 0.0f : 1.0f / df[k];
    }
    float t_ent = (float)en.t0;
    float q[3];
    for (int k = 0; k < 3; ++k) q[k] = of[k] + t_ent * df[k];
    if (en.kin >= 0) put(q, en.kin, en.side ? (float)Rd : 0.0f);
    uint32_t I, dep = 0, c[3];
    root_of<float>(q, up, v.R, c, I);
    uint4 r = ld_rec(rec, I);
    descend<float>(rec, q, up, I, dep, c, r);
    if (STATS) acc.descent += dep;
    float T = 1.0f, C[3] = {0.f, 0.f, 0.f};
    uint2 pay = ((const uint2*)v.pay)[I];
    for (uint32_t step = 0;; ++step) {
      if (step >= v.max_steps) { out.flags |= CVX_RAYFLAG_STEP_CAP; break; }
      float h = ldexpf(1.0f, -(int)dep);
      float best = BIGF;
      int kx = 0;
      float Xb = 0.f;
      for (int k = 0; k < 3; ++k) {
        if (par[k]) continue;
        float X = (float)(c[k] + (up[k] ? 1u : 0u)) * h;
        float tt = (X - of[k]) * idf[k];
        if (tt < best) { best = tt; kx = k; Xb = X; }
      }
      float len = (best - t_ent) * ldexpf(1.0f, (int)dep);
      len = len > 0.0f ? len : 0.0f;
      // every visited leaf is recorded: for a ray not within the face band of
      // a visited leaf the exact segment is positive even when it rounds to 0
      {
        float col[3], kap;
        decode8(pay, col, kap);
        float Tn = T * __expf(-kap * len);
        float a = T - Tn;
        for (int k = 0; k < 3; ++k) C[k] = __builtin_fma(a, col[k], C[k]);
        T = Tn;
        if (TRACE && n_rec < sk.cap) { sk.ids[n_rec] = I; if (sk.len32) sk.len32[n_rec] = len; if (sk.len64) sk.len64[n_rec] = len; }
        ++n_rec;
        if (use_stop && 1.0f - T >= v.alpha_stop) break;
      }
      const uint32_t ck = pick(c, kx);
      const bool upk = pick(up, kx);
      const uint32_t side_n = v.R << dep;
      if (upk ? (ck + 1u >= side_n) : (ck == 0u)) break;
      const uint32_t nc = upk ? ck + 1u : ck - 1u;
      uint32_t N;
      bool outer;
      if (dep == 0) {
        uint32_t stride = kx == 0 ? 1u : (kx == 1 ? v.R : v.R * v.R);
        N = upk ? I + stride : I - stride;
        outer = true;
      } else if ((ck & 1u) == (upk ? 0u : 1u)) {
        N = upk ? I + (1u << kx) : I - (1u << kx);
        outer = false;
      } else {
        N = kx == 0 ? r.y : (kx == 1 ? r.z : r.w);
        outer = true;
      }
      if (N == CVX_NONE) { out.flags |= CVX_RAYFLAG_BAD_LINK; break; }
      if (STATS) acc.outer += outer;
      put(c, kx, nc);
      uint4 rN = ld_rec(rec, N);
      I = N;
      r = rN;
      if (r.x & 1u) {
        uint32_t dN = (r.x >> 1) & 63u;
        if (dN < dep) {
          for (int k = 0; k < 3; ++k) c[k] >>= (dep - dN);
          dep = dN;
        }
      } else {
        for (int k = 0; k < 3; ++k) q[k] = of[k] + best * df[k];
        put(q, kx, Xb);
        uint32_t d0 = dep;
        descend<float>(rec, q, up, I, dep, c, r);
        if (STATS) acc.descent += dep - d0;
      }
      pay = ((const uint2*)v.pay)[I];
      t_ent = best > t_ent ? best : t_ent;
    }
    out.rgba[0] = C[0];
    out.rgba[1] = C[1];
    out.rgba[2] = C[2];
    out.rgba[3] = 1.0f - T;
    out.n = n_rec;
    if (STATS) acc.leaves += n_rec;
    return;
  }

  double inv[3];
  for (int k = 0; k < 3; ++k) inv[k] = 1.0 / d[k];
  double q[3];
  for (int k = 0; k < 3; ++k) q[k] = o[k] + en.t0 * d[k];
  if (en.kin >= 0) put(q, en.kin, en.side ? Rd : 0.0);
  for (int k = 0; k < 3; ++k) q[k] = q[k] < 0.0 ? 0.0 : (q[k] > Rd ? Rd : q[k]);
  uint32_t I, dep = 0, c[3];
  root_of<double>(q, up, v.R, c, I);
  uint4 r = ld_rec(rec, I);
  descend<double>(rec, q, up, I, dep, c, r);
  if (STATS) acc.descent += dep;

  // ---------------------------------------------------------------- FP64 plain
  if constexpr (VAR == (int)CVX_VARIANT_FP64_PLAIN) {
    double T = 1.0, C[3] = {0.0, 0.0, 0.0};
    double t_ent = en.t0;
    for (uint32_t step = 0;; ++step) {
      if (step >= v.max_steps) { out.flags |= CVX_RAYFLAG_STEP_CAP; break; }
      double h = ldexp(1.0, -(int)dep);
      double best = __builtin_inf();
      int kx = 0;
      for (int k = 0; k < 3; ++k) {
        if (d[k] == 0.0) continue;
        double X = (double)(c[k] + (up[k] ? 1u : 0u)) * h;
        double tt = (X - o[k]) * inv[k];
        if (tt < best) { best = tt; kx = k; }
      }
      double len = ldexp(best - t_ent, (int)dep);
      len = len > 0.0 ? len : 0.0;
      {
        double col[3], kap;
        if (v.fmt == CVX_LEAF_F64) {
          double4 p = ((const double4*)v.pay)[I];
          col[0] = p.x; col[1] = p.y; col[2] = p.z; kap = p.w;
        } else {
          uint2 p = ((const uint2*)v.pay)[I];
          col[0] = (double)(p.x & 0xffu) / 255.0;
          col[1] = (double)((p.x >> 8) & 0xffu) / 255.0;
          col[2] = (double)((p.x >> 16) & 0xffu) / 255.0;
          kap = (double)(float)__builtin_bit_cast(_Float16, (unsigned short)(p.y & 0xffffu));
        }
        double Tn = T * exp(-kap * len);
        double a = T - Tn;
        for (int k = 0; k < 3; ++k) C[k] = __builtin_fma(a, col[k], C[k]);
        T = Tn;
        if (TRACE && n_rec < sk.cap) { sk.ids[n_rec] = I; if (sk.len32) sk.len32[n_rec] = (float)len; if (sk.len64) sk.len64[n_rec] = len; }
        ++n_rec;
        if (use_stop && 1.0 - T >= (double)v.alpha_stop) break;
      }
      const uint32_t ck = pick(c, kx);
      const bool upk = pick(up, kx);
      const uint32_t side_n = v.R << dep;
      if (upk ? (ck + 1u >= side_n) : (ck == 0u)) break;
      const uint32_t nc = upk ? ck + 1u : ck - 1u;
      uint32_t N;
      bool outer;
      if (dep == 0) {
        uint32_t stride = kx == 0 ? 1u : (kx == 1 ? v.R : v.R * v.R);
        N = upk ? I + stride : I - stride;
        outer = true;
      } else if ((ck & 1u) == (upk ? 0u : 1u)) {
        N = upk ? I + (1u << kx) : I - (1u << kx);
        outer = false;
      } else {
        N = kx == 0 ? r.y : (kx == 1 ? r.z : r.w);
        outer = true;
      }
      if (N == CVX_NONE) { out.flags |= CVX_RAYFLAG_BAD_LINK; break; }
      if (STATS) acc.outer += outer;
      double X = (double)(upk ? nc : ck) * h;
      put(c, kx, nc);
      I = N;
      r = ld_rec(rec, N);
      if (r.x & 1u) {
        uint32_t dN = (r.x >> 1) & 63u;
        if (dN < dep) {
          for (int k = 0; k < 3; ++k) c[k] >>= (dep - dN);
          dep = dN;
        }
      } else {
        for (int k = 0; k < 3; ++k) q[k] = o[k] + best * d[k];
        put(q, kx, X);
        uint32_t d0 = dep;
        descend<double>(rec, q, up, I, dep, c, r);
        if (STATS) acc.descent += dep - d0;
      }
      t_ent = best > t_ent ? best : t_ent;
    }
    out.rgba[0] = C[0];
    out.rgba[1] = C[1];
    out.rgba[2] = C[2];
    out.rgba[3] = 1.0 - T;
    out.n = n_rec;
    if (STATS) acc.leaves += n_rec;
    return;
  }

  // ------------------------------------------------------------- FP32 rebased
  if constexpr (VAR == (int)CVX_VARIANT_FP32_REBASED) {
    float df[3], idf[3];
    bool par[3];
    for (int k = 0; k < 3; ++k) {
      par[k] = !(__builtin_fabs(d[k]) >= 0x1p-60);
      df[k] = (float)d[k];
      idf[k] = par[k] ? 0.0f : 1.0f / df[k];
    }
    // bound on |t| + |q| along the ray, for the rebase error bound
    const float tR = (float)(en.t1 + Rd + 1.0);
    float p[3];
    for (int k = 0; k < 3; ++k) p[k] = (float)((ldexp(q[k], (int)dep) - (double)c[k]) - 0.5);
    float ep = ldexpf(tR, (int)dep - 50) + 0x1p-24f;
    float T = 1.0f, C[3] = {0.f, 0.f, 0.f};
    uint2 pay = ((const uint2*)v.pay)[I];
    for (uint32_t step = 0;; ++step) {
      if (step >= v.max_steps) { out.flags |= CVX_RAYFLAG_STEP_CAP; break; }
      // exit face in cell-local FP32, with error bounds
      float tk[3], ek[3];
      for (int k = 0; k < 3; ++k) {
        if (par[k]) {
          tk[k] = BIGF;
          ek[k] = 0.0f;
        } else {
          float f = up[k] ? 0.5f : -0.5f;
          tk[k] = (f - p[k]) * idf[k];
          ek[k] = (ep + 0x1p-24f) * __builtin_fabsf(idf[k]) * 1.0001f +
                  0x1.81p-23f * __builtin_fabsf(tk[k]);
        }
      }
      int kx = tk[1] < tk[0] ? 1 : 0;
      if (tk[2] < pick(tk, kx)) kx = 2;
      const float tmin = pick(tk, kx), emin = pick(ek, kx);
      bool cert = true;
      for (int k = 0; k < 3; ++k) {
        float m = tk[k] - tmin;
        float need = (ek[k] + emin) * 1.0625f + 0x1p-22f * __builtin_fabsf(tk[k]);
        if (k != kx && !(m > need)) cert = false;
      }
      float len = tmin;
      float ekx = emin;
      bool force = false;
      if (!cert) {
        // FP64 decision from the exact face planes
        double h = ldexp(1.0, -(int)dep);
        double best = __builtin_inf();
        int kb = kx;
        for (int k = 0; k < 3; ++k) {
          if (d[k] == 0.0) continue;
          double X = (double)(c[k] + (up[k] ? 1u : 0u)) * h;
          double tt = (X - o[k]) * inv[k];
          if (tt < best) { best = tt; kb = k; }
        }
        if (pick(tk, kb) < BIGF) {
          len = pick(tk, kb);
          ekx = pick(ek, kb);
        }
        kx = kb;
        force = true;
        out.flags |= CVX_RAYFLAG_FP64_EXIT;
        if (STATS) acc.fp64_exit++;
      }
      len = len > 0.0f ? len : 0.0f;
      // every visited leaf is recorded: for a ray not within the face band of
      // a visited leaf the exact segment is positive even when it rounds to 0
      {
        float col[3], kap;
        decode8(pay, col, kap);
        float Tn = T * __expf(-kap * len);
        float a = T - Tn;
        for (int k = 0; k < 3; ++k) C[k] = __builtin_fma(a, col[k], C[k]);
        T = Tn;
        if (TRACE && n_rec < sk.cap) { sk.ids[n_rec] = I; if (sk.len32) sk.len32[n_rec] = len; if (sk.len64) sk.len64[n_rec] = len; }
        ++n_rec;
        if (use_stop && 1.0f - T >= v.alpha_stop) break;
      }
      const uint32_t ck = pick(c, kx);
      const bool upk = pick(up, kx);
      const uint32_t side_n = v.R << dep;
      if (upk ? (ck + 1u >= side_n) : (ck == 0u)) break;
      const uint32_t nc = upk ? ck + 1u : ck - 1u;
      uint32_t N;
      bool outer;
      if (dep == 0) {
        uint32_t stride = kx == 0 ? 1u : (kx == 1 ? v.R : v.R * v.R);
        N = upk ? I + stride : I - stride;
        outer = true;
      } else if ((ck & 1u) == (upk ? 0u : 1u)) {
        N = upk ? I + (1u << kx) : I - (1u << kx);
        outer = false;
      } else {
        N = kx == 0 ? r.y : (kx == 1 ? r.z : r.w);
        outer = true;
      }
      if (N == CVX_NONE) { out.flags |= CVX_RAYFLAG_BAD_LINK; break; }
      if (STATS) acc.outer += outer;
      uint4 rN = ld_rec(rec, N);
      uint2 payN = ((const uint2*)v.pay)[N];
      put(c, kx, nc);
      const bool leafN = rN.x & 1u;
      const uint32_t dN = leafN ? ((rN.x >> 1) & 63u) : dep;
      if (!leafN || force || ep > EP_MAX) {
        // FP64 rebase at the exactly known crossing plane
        double h = ldexp(1.0, -(int)dep);
        double X = (double)(upk ? nc : ck) * h;
        double tp = (X - pick(o, kx)) * pick(inv, kx);
        for (int k = 0; k < 3; ++k) q[k] = o[k] + tp * d[k];
        put(q, kx, X);
        if (dN < dep) {
          for (int k = 0; k < 3; ++k) c[k] >>= (dep - dN);
          dep = dN;
        }
        I = N;
        r = rN;
        if (!leafN) {
          uint32_t d0 = dep;
          descend<double>(rec, q, up, I, dep, c, r);
          payN = ((const uint2*)v.pay)[I];
          if (STATS) acc.descent += dep - d0;
        }
        for (int k = 0; k < 3; ++k)
          p[k] = (float)((ldexp(q[k], (int)dep) - (double)c[k]) - 0.5);
        ep = ldexpf(tR, (int)dep - 50) + 0x1p-24f;
        if (STATS) acc.rebase++;
      } else {
        // move to the exit point in the same-depth frame of the neighbour
        for (int k = 0; k < 3; ++k)
          p[k] = k == kx ? (upk ? -0.5f : 0.5f) : __builtin_fmaf(len, df[k], p[k]);
        ep = ep + ekx + len * 0x1p-23f + 0x1p-25f;
        if (dN < dep) {
          const uint32_t m = dep - dN;
          const float sc = ldexpf(1.0f, -(int)m);
          const uint32_t mask = (1u << m) - 1u;
          for (int k = 0; k < 3; ++k) {
            p[k] = ((float)(c[k] & mask) + (p[k] + 0.5f)) * sc - 0.5f;
            c[k] >>= m;
          }
          dep = dN;
          ep = ep * sc + 0x1p-23f;
        }
        I = N;
        r = rN;
      }
      pay = payN;
    }
    out.rgba[0] = C[0];
    out.rgba[1] = C[1];
    out.rgba[2] = C[2];
    out.rgba[3] = 1.0f - T;
    out.n = n_rec;
    if (STATS) acc.leaves += n_rec;
  }
}

template <int VAR, bool TRACE, bool STATS, bool OUT64>
__global__ __launch_bounds__(256) void k_cast(CastArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t total = a.hdr->total_work;
  const uint32_t nv = a.hdr->n_views;
  Acc acc = {0, 0, 0, 0, 0, 0};
  for (;;) {
    uint32_t w = 0;
    if (lane == 0) w = atomicAdd(&a.hdr->queue, 1u);
    w = __builtin_amdgcn_readfirstlane(__shfl(w, 0, 64));
    if ((uint64_t)w >= total) break;
    Out res;
    if constexpr (!TRACE) {
      int lo = 0, hi = (int)nv - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (a.views[mid].first_tile <= (uint64_t)w) lo = mid; else hi = mid - 1;
      }
      const DView& v = a.views[lo];
      uint64_t t = (uint64_t)w - v.first_tile;
      uint32_t tx = (uint32_t)(t % v.tiles_x), ty = (uint32_t)(t / v.tiles_x);
      uint32_t x = tx * a.tile_w + lane % a.tile_w, y = ty * a.tile_h + lane / a.tile_w;
      if (x < v.W && y < v.H) {
        Sink sk{nullptr, nullptr, nullptr, 0};
        cast_ray<VAR, false, STATS>(v, x, y, sk, acc, res);
        uint64_t pix = v.out_off + (uint64_t)y * v.W + x;
        if constexpr (OUT64) {
          double2* o2 = (double2*)a.out + 2 * pix;
          o2[0] = make_double2(res.rgba[0], res.rgba[1]);
          o2[1] = make_double2(res.rgba[2], res.rgba[3]);
        } else {
          ((float4*)a.out)[pix] = make_float4((float)res.rgba[0], (float)res.rgba[1],
                                              (float)res.rgba[2], (float)res.rgba[3]);
        }
      }
    } else {
      uint64_t ri = (uint64_t)w * 64u + lane;
      if (ri < a.hdr->n_rays) {
        uint64_t id = a.ray_ids[ri];
        uint32_t vi = (uint32_t)(id >> 32), pix = (uint32_t)(id & 0xffffffffu);
        a.n_leaves[ri] = 0;
        a.flags[ri] = CVX_RAYFLAG_BAD_LINK;
        if (vi < nv) {
          const DView& v = a.views[vi];
          if ((uint64_t)pix < (uint64_t)v.W * v.H) {
            Sink sk{a.leaf_ids + ri * a.max_leaves,
                    a.local_len ? a.local_len + ri * a.max_leaves : nullptr,
                    a.local_len64 ? a.local_len64 + ri * a.max_leaves : nullptr, a.max_leaves};
            cast_ray<VAR, TRACE, STATS>(v, pix % v.W, pix / v.W, sk, acc, res);
            a.n_leaves[ri] = res.n;
            a.flags[ri] = res.flags;
            ((float4*)a.trace_rgba)[ri] = make_float4((float)res.rgba[0], (float)res.rgba[1],
                                                      (float)res.rgba[2], (float)res.rgba[3]);
          }
        }
      }
    }
  }
  if constexpr (STATS) {
    uint32_t vals[6] = {acc.rays, acc.leaves, acc.outer, acc.descent, acc.fp64_exit, acc.rebase};
    for (int s = 0; s < 6; ++s) {
      uint32_t x = vals[s];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      if (lane == 0 && x) atomicAdd((unsigned long long*)&a.stats[s], (unsigned long long)x);
    }
  }
}

__global__ void k_reset(CastHeader* hdr) {
  if (threadIdx.x == 0 && blockIdx.x == 0) hdr->queue = 0u;
}

template <int VAR, bool TRACE, bool STATS, bool OUT64>
int launch_t(void* stream, const CastArgs& a, uint32_t wgs, uint32_t wg_size) {
  hipLaunchKernelGGL((k_cast<VAR, TRACE, STATS, OUT64>), dim3(wgs), dim3(wg_size), 0,
                     (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

template <int VAR>
int launch_v(void* stream, bool trace, bool stats, bool out64, const CastArgs& a, uint32_t wgs,
             uint32_t wg) {
  if (trace) return stats ? launch_t<VAR, true, true, false>(stream, a, wgs, wg)
                          : launch_t<VAR, true, false, false>(stream, a, wgs, wg);
  if (out64) return stats ? launch_t<VAR, false, true, true>(stream, a, wgs, wg)
                          : launch_t<VAR, false, false, true>(stream, a, wgs, wg);
  return stats ? launch_t<VAR, false, true, false>(stream, a, wgs, wg)
               : launch_t<VAR, false, false, false>(stream, a, wgs, wg);
}

}  // namespace

int launch_cast(void* stream, uint32_t variant, bool trace, bool stats, bool out_f64,
                const CastArgs& a, uint32_t workgroups, uint32_t wg_size) {
  switch (variant) {
    case CVX_VARIANT_FP32_REBASED:
      return launch_v<(int)CVX_VARIANT_FP32_REBASED>(stream, trace, stats, false, a, workgroups,
                                                     wg_size);
    case CVX_VARIANT_FP64_PLAIN:
      return launch_v<(int)CVX_VARIANT_FP64_PLAIN>(stream, trace, stats, out_f64, a, workgroups,
                                                   wg_size);
    case CVX_VARIANT_FP32_NAIVE:
      return launch_v<(int)CVX_VARIANT_FP32_NAIVE>(stream, trace, stats, false, a, workgroups,
                                                   wg_size);
    default:
      return (int)hipErrorInvalidValue;
  }
}

int launch_reset(void* stream, CastHeader* hdr) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, (hipStream_t)stream, hdr);
  return (int)hipGetLastError();
}

}  // namespace cvx

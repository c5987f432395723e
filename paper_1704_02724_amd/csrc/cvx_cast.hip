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
// All variants share the integer bookkeeping: node id, depth and the integer
// coordinates of the cell at that depth, which make every face plane an exact
// dyadic.  Per-axis state lives in V3 structs (never in arrays indexed by a
// run-time axis) so that it stays in registers.
//  FP32_REBASED  cell-local FP32 DDA with certified decisions (cast_fp32).
//  FP64_PLAIN    canvas-global FP64: exit t from the exact face planes each
//                step, FP64 compositing.  The GPU baseline.
//  FP32_NAIVE    canvas-global FP32 (the paper's "canvas coordinate"
//                traversal that drifts at depth); kept to show the failure.
//  FP32_CELL_LOCAL  the paper's own cell-local FP32 traversal (Sec. 6.2),
//                uncertified; the subject of its error analysis (Sec. 6.3).
//  FP16_CELL_LOCAL  the same traversal in IEEE half precision, the case the
//                end of Sec. 6.3 argues would suffice.
#include <hip/hip_runtime.h>

#include <mutex>

#include "cvx_internal.h"

#ifndef CVX_CAST32_WAVES
#define CVX_CAST32_WAVES 8
#endif
#ifndef CVX_CAST32R_WAVES
#define CVX_CAST32R_WAVES 7
#endif

namespace cvx {

namespace {

constexpr float BIGF = 1e30f;

template <class T>
struct V3 {
  T x, y, z;
};

// Component k of v; k is a run-time axis (compiles to selects) or a constant.
// v is taken by value: a select between loads of one object would otherwise
// be folded into a variable-offset load, which forces the struct into memory.
template <class T>
__device__ __forceinline__ T get(V3<T> v, int k) {
  T r = v.x;
  r = k == 1 ? v.y : r;
  r = k == 2 ? v.z : r;
  return r;
}
template <class T>
__device__ __forceinline__ void set(V3<T>& v, int k, T a) {
  const V3<T> u = v;
  v = V3<T>{k == 0 ? a : u.x, k == 1 ? a : u.y, k == 2 ? a : u.z};
}

// Per-lane boolean logic on wavefront lane masks: the compare results are
// combined with scalar instructions instead of being materialised as 0/1 in
// vector registers (the compiler does the latter for some select shapes).
__device__ __forceinline__ uint64_t lanes(bool b) { return __builtin_amdgcn_ballot_w64(b); }
__device__ __forceinline__ bool lane(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// 2 c + b for a per-lane bit given as a lane mask: one add with the mask as
// carry-in (v_addc_co_u32); the compiler would emit a select and a shift-or.
// The carry-out is written to a scratch SGPR pair and not used.
__device__ __forceinline__ uint32_t twice_plus(uint32_t c, uint64_t b) {
  uint32_t r;
  uint64_t co;
  asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(r), "=s"(co) : "v"(c), "s"(b));
  return r;
}

// Cell indices between true and direction-normalised form (an involution):
// component k xor all ones when the ray travels down axis k.
__device__ __forceinline__ V3<uint32_t> flip(V3<uint32_t> c, const V3<bool>& up) {
  return V3<uint32_t>{c.x ^ (up.x ? 0u : ~0u), c.y ^ (up.y ? 0u : ~0u), c.z ^ (up.z ? 0u : ~0u)};
}

struct Acc {
  uint32_t rays, leaves, outer, descent, fp64_exit, rebase;
  uint64_t steps, slots;  // loop iterations of the lanes; 64 x the longest lane per tile
};

struct Out {
  double rgba[4];
  double T;        // FP32_REBASED: the transmittance (a chord piece's, when split)
  double end[3];   // trace mode: the exit point of the last leaf as the variant computed it
  uint32_t flags;
  uint32_t n;
  uint32_t steps;  // loop iterations of this ray
};

// Trace sink: records (leaf, l) pairs when tracing is on.
struct Sink {
  uint32_t* ids;
  float* len32;
  double* len64;
  uint32_t cap;
};

__device__ __forceinline__ void record(Sink& sk, uint32_t n, uint32_t I, double len) {
  if (n < sk.cap) {
    sk.ids[n] = I;
    if (sk.len32) sk.len32[n] = (float)len;
    if (sk.len64) sk.len64[n] = len;
  }
}

// FP64 reciprocal square root and reciprocal: the hardware estimate
// (v_rsq_f64, v_rcp_f64) refined by two Newton steps in FMA form, within an
// ulp or two of the correctly rounded value, instead of the IEEE square root
// and division sequences (several times as many half-rate instructions).
// rcp_nr(x) for |x| < 2^-1000 (zero included) is +-inf, as 1/x overflows.
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;  // exact
  for (int i = 0; i < 2; ++i) y = __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
  return y;
}
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  for (int i = 0; i < 2; ++i) r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
  return __builtin_fabs(x) < 0x1p-1000 ? __builtin_copysign(__builtin_inf(), x) : r;
}

// FP64 unit direction of pixel (x, y) in the public convention
// (normalize(fwd + u right + v up), u and v from the pixel centre), no
// contraction.  The divisions by the image size are products with the
// view's 2/W and 2/H (each rounded once) and the normalisation multiplies by
// a reciprocal square root of the squared norm: each component stays within
// a few FP64 ulp of the convention's division form, far inside the 1e-12
// band in which crossings count as ambiguous.
__device__ __forceinline__ V3<double> ray_dir(const DView& v, uint32_t x, uint32_t y) {
#pragma clang fp contract(off)
  double u = (((double)x + 0.5) * v.two_w - 1.0) * v.tan_x;
  double w = (1.0 - ((double)y + 0.5) * v.two_h) * v.tan_y;
  double d[3], n2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    d[k] = v.fwd[k] + u * v.right[k];
    d[k] = d[k] + w * v.up[k];
    n2 += d[k] * d[k];
  }
  const double rn = rsq_nr(n2);
  return V3<double>{d[0] * rn, d[1] * rn, d[2] * rn};
}

struct Entry {
  double t0, t1;
  int kin, side;
  bool hit;
};

// Slab test of the ray against the canvas box [0, R]^3 (FP64), with the
// ray's reciprocal direction inv (rcp_nr, one per axis per ray).
__device__ __forceinline__ Entry canvas_entry(const V3<double>& o, const V3<double>& d,
                                              const V3<double>& inv, double Rd) {
  Entry e;
  double tin = -__builtin_inf(), tout = __builtin_inf();
  int kin = -1, side = 0;
  bool miss = false;
  for (int k = 0; k < 3; ++k) {
    const double dk = get(d, k), ok = get(o, k);
    if (dk != 0.0) {
      const double ik = get(inv, k);
      double ta = (0.0 - ok) * ik, tb = (Rd - ok) * ik;
      double lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
      if (lo > tin) {
        tin = lo;
        kin = k;
        side = dk > 0.0 ? 0 : 1;
      }
      if (hi < tout) tout = hi;
    } else if (ok < 0.0 || ok > Rd) {
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

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(1))) u32x4_t* grec_t;
typedef const __attribute__((address_space(1))) u32x2_t* gpay_t;

// Pool loads through the global address space (the pointers come from the
// view table, so the compiler would otherwise emit flat loads).
__device__ __forceinline__ uint4 ld_rec(const void* rec, uint32_t i) {
  const u32x4_t x = ((grec_t)rec)[i];
  return make_uint4(x.x, x.y, x.z, x.w);
}
__device__ __forceinline__ uint2 ld_pay(const void* pay, uint32_t i) {
  const u32x2_t x = ((gpay_t)pay)[i];
  return make_uint2(x.x, x.y);
}
// The same with a 32-bit byte offset from the (uniform) base, for pools of at
// most 2^28 nodes: the loads take the scalar-base form and the per-step
// 64-bit address arithmetic goes away.
template <bool SMALL>
__device__ __forceinline__ uint4 ld_rec_t(const void* rec, uint32_t i) {
  if constexpr (!SMALL) return ld_rec(rec, i);
  const u32x4_t x = *(grec_t)((const __attribute__((address_space(1))) char*)rec + (i << 4));
  return make_uint4(x.x, x.y, x.z, x.w);
}
template <bool SMALL>
__device__ __forceinline__ uint2 ld_pay_t(const void* pay, uint32_t i) {
  if constexpr (!SMALL) return ld_pay(pay, i);
  const u32x2_t x = *(gpay_t)((const __attribute__((address_space(1))) char*)pay + (i << 3));
  return make_uint2(x.x, x.y);
}

// Descend from the current cell (r refined) to the leaf containing q; on a
// mid-plane the child on the side the ray moves into is taken.  Returns false
// (and stops) if a child index falls outside the pool.
template <class Real>
__device__ __forceinline__ bool descend(const void* rec, uint32_t n_nodes, const V3<Real>& q,
                                        const V3<bool>& up, uint32_t& I, uint32_t& dep,
                                        V3<uint32_t>& c, uint4& r) {
  while (!(r.x & 1u)) {
    if (r.x >= n_nodes - 7u) return false;
    const Real h = (Real)ldexp(1.0, -(int)dep);
    uint32_t oct = 0;
    for (int k = 0; k < 3; ++k) {
      const Real mid = ((Real)get(c, k) + (Real)0.5) * h;
      const Real qk = get(q, k);
      const uint32_t b = (qk > mid) || (qk == mid && get(up, k));
      oct |= b << k;
      set(c, k, 2u * get(c, k) + b);
    }
    I = r.x + oct;
    ++dep;
    r = ld_rec(rec, I);
  }
  return true;
}

// Integer point location.  The FP64 point q (canvas units, inside [0, R]^3)
// maps to the coordinates of its cell at the deepest level D:
//   C_k = floor(q_k 2^D), one less when q_k 2^D is an integer and the ray
//   moves down axis k,
// clamped to the canvas.  q_k 2^D and its floor are exact in FP64 (R 2^D <=
// 2^30).  For a cell containing q, the child on axis k is the upper one iff
// q_k > mid or (q_k = mid and the ray moves up axis k) (ties go to the side
// the ray moves into); with C clamped to the cell this is the matching bit
// of C, at every level.  So a descent is one clamp and then integer work.
__device__ __forceinline__ V3<uint32_t> deep_coords(const V3<double>& q, const V3<bool>& up,
                                                    uint32_t R, uint32_t D) {
  V3<uint32_t> C;
  const int32_t hi = (int32_t)((R << D) - 1u);
  for (int k = 0; k < 3; ++k) {
    const double Q = ldexp(get(q, k), (int)D);
    const double f = floor(Q);
    int32_t n = (int32_t)f;
    n -= (Q == f && !get(up, k)) ? 1 : 0;
    n = n < 0 ? 0 : (n > hi ? hi : n);
    set(C, k, (uint32_t)n);
  }
  return C;
}

// Descend from the current cell (I, dep, c; record r) to the leaf holding the
// deep coordinates C.  Returns false (and stops) if a child index falls
// outside the pool.
__device__ __forceinline__ bool descend_int(const void* rec, uint32_t n_nodes, V3<uint32_t> C,
                                            uint32_t D, uint32_t& I, uint32_t& dep,
                                            V3<uint32_t>& c, uint4& r) {
  if (r.x & 1u) return true;
  for (int k = 0; k < 3; ++k) {
    const uint32_t lo = get(c, k) << (D - dep);
    const uint32_t hi = lo + ((1u << (D - dep)) - 1u);
    const uint32_t ck = get(C, k);
    set(C, k, ck < lo ? lo : (ck > hi ? hi : ck));
  }
  while (!(r.x & 1u)) {
    if (r.x >= n_nodes - 7u) return false;
    const uint32_t sh = D - dep - 1u;
    uint32_t oct = 0;
    for (int k = 0; k < 3; ++k) {
      const uint32_t b = (get(C, k) >> sh) & 1u;
      oct |= b << k;
      set(c, k, 2u * get(c, k) + b);
    }
    I = r.x + oct;
    ++dep;
    r = ld_rec(rec, I);
  }
  return true;
}

// Cell of a ray start: through the top-level table when the view has one
// (the node of depth <= L covering the depth-L cell of C), else the root.
__device__ __forceinline__ void locate_top(const DView& v, const V3<uint32_t>& C, uint32_t& I,
                                           uint32_t& dep, V3<uint32_t>& c, uint4& r) {
  const uint32_t D = v.max_depth;
  if (v.top_depth) {
    const uint32_t L = v.top_depth, side = v.R << L;
    const uint32_t x = C.x >> (D - L), y = C.y >> (D - L), z = C.z >> (D - L);
    I = v.top[x + side * (y + side * z)];
    r = ld_rec(v.rec, I);
    dep = (r.x & 1u) ? ((r.x >> 1) & 63u) : L;
  } else {
    I = (C.x >> D) + v.R * ((C.y >> D) + v.R * (C.z >> D));
    r = ld_rec(v.rec, I);
    dep = 0;
  }
  c = V3<uint32_t>{C.x >> (D - dep), C.y >> (D - dep), C.z >> (D - dep)};
}

// First cell of a ray at its FP64 start point q: the view's shared eye leaf
// when the view has one (every ray then starts at q = eye, off every plane of
// the deepest grid, so all of them locate the same leaf), else the
// top-level-table (or root-array) cell above q; a refined cell is descended
// by the caller.
__device__ __forceinline__ void start_leaf(const DView& v, const V3<double>& q, const V3<bool>& up,
                                           uint32_t& I, uint32_t& dep, V3<uint32_t>& c,
                                           uint4& r, bool shared = true) {
  if (shared && v.start_ok) {
    I = v.start_node;
    dep = v.start_dep;
    c = V3<uint32_t>{v.start_c[0], v.start_c[1], v.start_c[2]};
    r = ld_rec(v.rec, I);
  } else {
    locate_top(v, deep_coords(q, up, v.R, v.max_depth), I, dep, c, r);
  }
}

// Root cell containing q (ties go to the side the ray moves into).
template <class Real>
__device__ __forceinline__ void root_of(const V3<Real>& q, const V3<bool>& up, uint32_t R,
                                        V3<uint32_t>& c, uint32_t& I) {
  for (int k = 0; k < 3; ++k) {
    const Real qk = get(q, k);
    const Real f = floor(qk);
    int n = (int)f;
    if (qk == f && !get(up, k)) n -= 1;
    n = n < 0 ? 0 : n;
    n = n > (int)R - 1 ? (int)R - 1 : n;
    set(c, k, (uint32_t)n);
  }
  I = c.x + R * (c.y + R * c.z);
}

// Neighbour across the exit face on axis kx: the sibling (inner face, index
// arithmetic), the next root (root array), or the stored outer-face link.
struct Move {
  uint32_t N, nc;
  bool at_edge, outer;
};

__device__ __forceinline__ Move neighbour(const DView& v, uint32_t I, const uint4 r, uint32_t dep,
                                          uint32_t ck, bool upk, int kx) {
  Move m;
  m.at_edge = upk ? (ck + 1u >= (v.R << dep)) : (ck == 0u);
  m.nc = upk ? ck + 1u : ck - 1u;
  const bool root = dep == 0;
  const bool inner = !root && ((ck & 1u) == (upk ? 0u : 1u));
  uint32_t rstride = 1u;
  rstride = kx == 1 ? v.R : rstride;
  rstride = kx == 2 ? v.R * v.R : rstride;
  const uint32_t stride = root ? rstride : (1u << kx);
  const uint32_t sib = upk ? I + stride : I - stride;
  uint32_t link = r.y;
  link = kx == 1 ? r.z : link;
  link = kx == 2 ? r.w : link;
  m.N = (root || inner) ? sib : link;
  m.outer = !inner;
  return m;
}

// An empty asm the compiler must assume rewrites x.  Loads and arithmetic
// that depend on the result cannot be hoisted out of the loop holding it, so
// the rare FP64 paths re-read their loop-invariant inputs (eye, view basis)
// there instead of pinning them in registers for the whole traversal.
template <class T>
__device__ __forceinline__ T opaque(T x) {
  asm volatile("" : "+v"(x));
  return x;
}

// The same for a wavefront-uniform value held in a scalar register.
__device__ __forceinline__ uint32_t opaque_s(uint32_t x) {
  asm volatile("" : "+s"(x));
  return x;
}

__device__ __forceinline__ float kappa_of(uint2 p) {
  return (float)__builtin_bit_cast(_Float16, (unsigned short)(p.y & 0xffffu));
}

// ----------------------------------------------------------------------------
// FP32_REBASED: cell-local FP32 traversal (Sec. 6.1-6.2) as a certified DDA.
//
// After a rebase at the entry point p0 (ray parameter te) of a cell, lengths
// are measured in "base units", the edge of a cell of depth db (a few levels
// below the current leaf), from p0: s = (t - te) / h_db.  For every axis k the
// face plane of the current leaf that lies ahead of the ray (its far plane in
// the travel direction) is held as an exact integer offset N_k, in base cells,
// from the far plane of the rebase cell, whose s-value S0_k was computed in
// FP64.  The far plane's s-value is S_k = S0_k + N_k / |d_k| with a constant
// error bound (no drift with the number of steps, unlike the per-step update
// analysed in Sec. 6.3):
//   |S_k - exact| <= ALPHA (S0_k + |N_k| / |d_k|) + beta,  beta = 2^(db-50) tR,
// ALPHA covering the FP32 roundings of S0, 1/|d|, N and the fused update.
// Exit = argmin S_k, certified when the lower bounds of the other two exceed
// its upper bound; otherwise the FP64 face planes decide.  A same-depth
// step adds the cell width w = 2^(db-dep) to N on the exit axis; a step into a
// coarser leaf adds the integer distance to its far planes; a refined cell is
// descended one level per iteration by comparing the entry s with the
// mid-plane s-values (certified likewise).  FP64 rebuilds the state
// ("rebase") only at the ray's start, after an FP64 decision, or when a
// descent goes below db or cannot be certified.
// ----------------------------------------------------------------------------
constexpr float ALPHA = 0x1p-21f;
// certification bound per plane value: 1.0625 (ALPHA G + beta) plus 2^-23 G
// for the FP32 rounding of the comparison (G >= |value|), folded into one fma
constexpr float ALPHA_C = 0x1p-21f * 1.0625f + 0x1p-23f;
constexpr float BETA_C = 1.0625f;
constexpr uint32_t DB_MARGIN = 8;

// Per-lane LDS slot holding the FP64 eye, direction and reciprocal direction
// of the lane's ray, [9][blockDim.x] doubles (component-major, so lanes read
// consecutive words).  The FP32 traversal needs them only on its rare FP64
// paths; keeping them here instead of in registers raises the number of
// resident wavefronts.
extern __shared__ double s_ray[];

typedef __attribute__((address_space(3))) double lds_f64;

struct RaySlot {
  lds_f64* p;  // this lane's first component
  uint32_t stride;
  __device__ __forceinline__ void put(const V3<double>& o, const V3<double>& d,
                                      const V3<double>& inv) const {
    p[0] = o.x; p[stride] = o.y; p[2 * stride] = o.z;
    p[3 * stride] = d.x; p[4 * stride] = d.y; p[5 * stride] = d.z;
    p[6 * stride] = inv.x; p[7 * stride] = inv.y; p[8 * stride] = inv.z;
  }
  // component j (0-2 eye, 3-5 direction, 6-8 reciprocal direction), read
  // through an opaque pointer so the load stays on the rare path that needs it
  __device__ __forceinline__ double at(int j) const { return opaque(p)[j * stride]; }
};

// Work of one wavefront in the refilling render kernel: the rays of up to
// `item_tiles` consecutive tiles of one view, numbered 64 per tile.  A lane
// whose ray ends waits until at least `refill_min` lanes of the wavefront
// wait; then each waiting lane takes the next ray of the item that is not
// taken yet (a wavefront ballot of the waiting lanes gives each its rank).
struct RefillJob {
  float4* out;
  uint64_t first_tile;  // the item's first tile within its view
  uint32_t n_rays;      // 64 x its tiles
  uint32_t tile_w, tile_h;
  uint32_t refill_min;
};

// FP32_REBASED traversal of one lane: one ray (REFILL = false: o, d, inv,
// en, up describe it) or, REFILL = true, the rays a RefillJob hands out one
// after another, each written to its pixel when it ends.  The per-ray
// arithmetic is the same in both, so both give the same pixels.
// SPLIT = true: the ray's chord is cut at ray parameter t_end (the end of a
// chord piece; infinity for the last piece): the leaf holding t_end
// contributes only the part before it, decided like an exit (certified, else
// in FP64 from the exact exit plane), and the piece ends there; a piece that
// does not start at the canvas entry locates its first leaf from its start
// point (shared_start = false: not through the view's shared eye leaf).
template <bool TRACE, bool STATS, bool SMALL, bool REFILL = false, bool SPLIT = false>
__device__ void cast_fp32(const DView& v, const RaySlot slot, const V3<double>& o_in,
                          const V3<double>& d_in, const V3<double>& inv_in, const Entry& en_in,
                          const V3<bool>& up_in, Sink sk, Acc& acc, Out& out,
                          const RefillJob* job = nullptr, double t_end = 0.0,
                          bool shared_start = true) {
  static_assert(!(REFILL && SPLIT), "chord pieces are traced one per lane");
  const void* rec = v.rec;
  const void* payp = v.pay;
  const bool use_stop = v.alpha_stop < 1.0f;
  V3<float> tD;
  bool anypar = false;
  float tR = 0.0f;
  V3<bool> up;
  V3<double> q;
  uint32_t I = 0, dep = 0;
  // cell indices at depth dep, direction-normalised: c_k xor all ones when
  // the ray travels down axis k, so that the next cell along the ray is
  // always c_k + 1 and an arithmetic shift right gives the parent's index
  // (R 2^max_depth <= 2^30: the sign bit is the direction)
  V3<uint32_t> c;
  uint4 r;
  uint2 pay = make_uint2(0u, 0u);
  uint32_t db = 0, w = 1;
  V3<float> S0{0.f, 0.f, 0.f};
  V3<int32_t> Nk{0, 0, 0};
  float s_ent = 0.0f, e_ent = 0.0f, betac = 0.0f;  // betac = BETA_C beta
  bool bad = false;  // a node index outside the pool (never for a validated pool)
  double te_last = 0.0;  // trace mode: ray parameter of the last rebase
  float T = 1.0f;
  V3<float> C{0.f, 0.f, 0.f};
  uint32_t n_rec = 0;
  // bit (1, 2 or 4) of the axis of the face the current cell was entered
  // through; 0 where the ray started inside the canvas
  uint32_t kbe = 0;
  uint32_t ub = 0;
  uint32_t step = 0;
  uint32_t end_Nn = 0, end_nc = 0, end_dep = 0;  // the move the ray ended on
  // the ray ended at the canvas boundary or the opacity stop; it leaves the
  // loop at the top of the next iteration (one exit, so the loop-carried
  // values need no copies for a second one)
  bool done = false;
  // SPLIT: s-value of the piece's end and its error bound (BIGF: no end)
  float s_end = BIGF, e_end = 0.0f;
  // FP64 rebuild of the base frame at ray parameter te (q = FP64 point); the
  // current cell I is descended first when it is refined.
  auto rebase = [&](double te) __attribute__((always_inline)) {
    if (TRACE) te_last = te;
    const uint32_t d0 = dep;
    V3<uint32_t> cr = flip(c, up);  // true indices
    bad = bad || !descend_int(rec, v.n_nodes, deep_coords(q, up, v.R, v.max_depth), v.max_depth,
                              I, dep, cr, r);
    if (STATS) acc.descent += dep - d0;
    pay = ld_pay_t<SMALL>(payp, I);
    db = dep + DB_MARGIN < v.max_depth ? dep + DB_MARGIN : (v.max_depth > dep ? v.max_depth : dep);
    w = 1u << (db - dep);
    const double hd = ldexp(1.0, -(int)dep);
    // rolled: one FP64 plane live at a time; the plane's parameter uses the
    // ray's reciprocal direction (a few FP64 ulp, inside the rebase term of
    // the bound)
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
      const double X = (double)get(cr, k) * hd + (get(up, k) ? hd : 0.0);  // exact
      const double Tk = (X - slot.at(k)) * slot.at(6 + k);
      set(S0, k, get(tD, k) == 0.0f ? BIGF : (float)ldexp(Tk - te, (int)db));
    }
    c = flip(cr, up);
    Nk = V3<int32_t>{0, 0, 0};
    s_ent = 0.0f;
    const float beta = ldexpf(tR, (int)db - 50);
    e_ent = beta;
    betac = beta * BETA_C;
    if constexpr (SPLIT) {
      // (t_end - te) 2^db rounded to FP32 (2^-24 relative) after an FP64
      // difference within beta
      const bool has_end = t_end < __builtin_inf();
      s_end = has_end ? (float)ldexp(t_end - te, (int)db) : BIGF;
      e_end = has_end ? beta + __builtin_fabsf(s_end) * 0x1p-23f : 0.0f;
    }
    if (STATS) acc.rebase++;
  };
  // ray start: the FP64 entry point, the first leaf and the first frame (Rd =
  // the canvas side R in FP64)
  auto begin = [&](const V3<double>& o, const V3<double>& d, const V3<double>& inv,
                   const Entry& en, const V3<bool>& up_, double Rd) __attribute__((always_inline)) {
    slot.put(o, d, inv);
    for (int k = 0; k < 3; ++k) {
      const double dk = get(d, k);
      set(tD, k, __builtin_fabs(dk) >= 0x1p-60 ? 1.0f / __builtin_fabsf((float)dk) : 0.0f);
    }
    anypar = tD.x == 0.0f || tD.y == 0.0f || tD.z == 0.0f;
    tR = (float)(en.t1 + Rd + 1.0);
    up = up_;
    // first leaf: the view's shared eye leaf, else FP64 point location from
    // the top-level table or the root array (descended to the leaf by the
    // rebase)
    for (int k = 0; k < 3; ++k) {
      double qk = get(o, k) + en.t0 * get(d, k);
      if (k == en.kin) qk = en.side ? Rd : 0.0;
      set(q, k, qk < 0.0 ? 0.0 : (qk > Rd ? Rd : qk));
    }
    dep = 0;
    start_leaf(v, q, up, I, dep, c, r, shared_start);
    c = flip(c, up);
    if (STATS) acc.descent += dep;
    pay = make_uint2(0u, 0u);
    db = 0;
    w = 1;
    bad = false;
    te_last = 0.0;
    rebase(en.t0);
    T = 1.0f;
    C = V3<float>{0.f, 0.f, 0.f};
    n_rec = 0;
    kbe = en.kin < 0 ? 0u : 1u << en.kin;
    // travel direction bits (x | y<<1 | z<<2) in one opaque register: the
    // exit-axis bit is one bit-field extract, not a chain of selects
    ub = opaque((up.x ? 1u : 0u) | (up.y ? 2u : 0u) | (up.z ? 4u : 0u));
    step = 0;
    end_Nn = end_nc = end_dep = 0;
    done = false;
  };
  // flags, colour and counts of the ray that ended
  auto finish = [&]() __attribute__((always_inline)) {
    if (bad)
      out.flags |= CVX_RAYFLAG_BAD_LINK;
    else if (!done && step >= v.max_steps)
      out.flags |= CVX_RAYFLAG_STEP_CAP;
    else if (end_Nn >= v.n_nodes && end_nc < (v.R << end_dep))
      out.flags |= CVX_RAYFLAG_BAD_LINK;  // a null link inside the canvas
    const float k255 = 1.0f / 255.0f;
    out.rgba[0] = C.x * k255;
    out.rgba[1] = C.y * k255;
    out.rgba[2] = C.z * k255;
    out.rgba[3] = 1.0f - T;
    out.T = T;
    out.n = n_rec;
    out.steps = done ? step : step + 1;  // a ray that ended left one iteration later
    if (STATS) acc.leaves += n_rec;
  };
  // REFILL: the pixel of the lane's current ray; starting ray i of the job
  // (false when its pixel lies outside the view, or when the ray misses the
  // canvas: its pixel is then written as zero)
  uint32_t px = 0, py = 0;
  auto write_pixel = [&]() __attribute__((always_inline)) {
    job->out[v.out_off + (uint64_t)py * v.W + px] = make_float4(
        (float)out.rgba[0], (float)out.rgba[1], (float)out.rgba[2], (float)out.rgba[3]);
  };
  auto begin_job_ray = [&](uint32_t i) __attribute__((always_inline)) -> bool {
    const uint64_t t = job->first_tile + i / 64u;
    const uint32_t l = i % 64u;
    px = (uint32_t)(t % v.tiles_x) * job->tile_w + l % job->tile_w;
    py = (uint32_t)(t / v.tiles_x) * job->tile_h + l / job->tile_w;
    if (px >= v.W || py >= v.H) return false;
    // the view's sizes pass an opaque barrier here, so that their FP64
    // conversions stay on this path instead of living (in vector registers)
    // through the traversal loop
    DView vr = v;
    vr.W = opaque_s(v.W);
    vr.H = opaque_s(v.H);
    const double Rd = (double)opaque_s(v.R);
    const V3<double> d = ray_dir(vr, px, py);
    const V3<double> o{v.o[0], v.o[1], v.o[2]};
    const V3<double> inv{rcp_nr(d.x), rcp_nr(d.y), rcp_nr(d.z)};
    const Entry en = canvas_entry(o, d, inv, Rd);
    out.rgba[0] = out.rgba[1] = out.rgba[2] = out.rgba[3] = 0.0;
    out.flags = 0;
    if (!en.hit) {
      write_pixel();
      return false;
    }
    begin(o, d, inv, en, V3<bool>{d.x > 0.0, d.y > 0.0, d.z > 0.0}, Rd);
    return true;
  };
  bool alive = true;
  uint32_t next = 64;     // REFILL: rays of the job handed out so far
  uint32_t wait_for = 0;  // REFILL: waiting lanes that end a traversal round
  if constexpr (REFILL) {
    alive = begin_job_ray(threadIdx.x & 63u);
    wait_for = job->refill_min;
  } else {
    begin(o_in, d_in, inv_in, en_in, up_in, (double)v.R);
  }
  // REFILL: rounds of traversal; a round ends when wait_for lanes wait, then
  // the waiting lanes take the job's next rays (ranked by a ballot), and once
  // none is left the last round runs until every lane waits.  The ray set-up
  // stays out of the traversal loop.
  for (;;) {
  for (;; ++step) {
    if constexpr (REFILL) {
      // every lane of the wavefront is here (uniform count)
      if ((uint32_t)__popcll(__ballot(!alive)) >= wait_for) break;
      if (!alive) continue;
    }
    if (step >= v.max_steps || bad || done) {
      if constexpr (!REFILL) break;
      finish();
      write_pixel();
      alive = false;
      continue;
    }
    // s-values of the far planes (leaf) or of the mid-planes (refined cell)
    // and their error bounds; a refined cell's mid-plane lies half a cell
    // before its far plane
    const bool leaf = r.x & 1u;
    const uint32_t half = w >> 1;
    const int32_t off = (int32_t)(half & ~(uint32_t)(-(int32_t)(r.x & 1u)));  // 0 for a leaf
    V3<float> S, eb;
    for (int k = 0; k < 3; ++k) {
      const float Nf = (float)(get(Nk, k) - off);
      set(S, k, __builtin_fmaf(Nf, get(tD, k), get(S0, k)));
      set(eb, k, __builtin_fmaf(ALPHA_C, __builtin_fmaf(__builtin_fabsf(Nf), get(tD, k), get(S0, k)),
                                betac));
    }
    bool need64 = false;
    if (!leaf) {
      // ---- refined cell entered through its near face on axis kbe: one level.
      // A refined cell is only reached by a leaf step (kbe != 0), and its
      // neighbours are of the same depth, so on axis kbe the entry value s_ent
      // and the mid-plane differ by exactly half a cell in N (>= 1 base cell,
      // far above the bounds): the entry side of that axis needs no test.
      need64 = w < 2u || anypar;
      if (r.x >= v.n_nodes - 7u) {  // ends the ray at the top of the loop
        bad = true;
        continue;
      }
      uint32_t oct = 0;
      for (int k = 0; k < 3; ++k) {
        const float diff = s_ent - get(S, k);
        const bool far = diff >= 0.0f;
        const bool sure = __builtin_fabsf(diff) > e_ent + get(eb, k);
        need64 = need64 || !sure;
        const uint32_t b = (get(up, k) == far) ? 1u : 0u;  // the child's octant bit
        oct |= b << k;
        set(Nk, k, get(Nk, k) - (far ? 0 : (int32_t)half));
        set(c, k, twice_plus(get(c, k), lanes(far)));  // normalised: the far child is next
      }
      if (!need64) {
        I = r.x + oct;
        ++dep;
        w = half;
        r = ld_rec_t<SMALL>(rec, I);
        pay = ld_pay_t<SMALL>(payp, I);
        if (STATS) acc.descent++;
        continue;
      }
      // undo the speculative update; the FP64 rebase descends from here
      for (int k = 0; k < 3; ++k) {
        const uint32_t ck = get(c, k);
        const bool far = (ck & 1u) != 0u;
        set(Nk, k, get(Nk, k) + (far ? 0 : (int32_t)half));
        set(c, k, (uint32_t)((int32_t)ck >> 1));
      }
    } else {
      // ---- leaf: exit face, certified against the error bounds
      const float Smin = __builtin_fminf(S.x, __builtin_fminf(S.y, S.z));
      // exit axis (ties to the lower axis) as its bit kbit (1, 2, 4), also
      // held one-hot as lane masks mx, my (z when neither) for the selects
      // below
      const uint64_t bx = lanes(S.x == Smin);
      bool mx = lane(bx);
      bool my = lane(lanes(S.y == Smin) & ~bx);
      uint32_t kbit = mx ? 1u : (my ? 2u : 4u);
      // ---- neighbour across the exit face: sibling, next root or G_3 link.
      // Its record load is issued as soon as the exit axis is known (again
      // after an FP64 decision), so that its latency overlaps the
      // certification and the composite instead of stalling the move.
      uint32_t nc = 0;  // normalised index of the next cell on the exit axis
      bool upk = false, inner = false;
      auto neighbour = [&](uint4 rr) __attribute__((always_inline)) -> uint32_t {
        const uint32_t ck = mx ? c.x : (my ? c.y : c.z);  // normalised
        upk = (ub & kbit) != 0u;
        nc = ck + 1u;
        const bool root = dep == 0;
        // the sibling lies across the face when the normalised index is even
        // (the cell is even going up, odd going down); siblings differ in
        // the exit axis's octant bit only
        inner = !root && (ck & 1u) == 0u;
        uint32_t sib = I ^ kbit;
        if (root) {
          // root array (rare): kept as a branch, not flattened into selects
          asm volatile("");
          const uint32_t ncr = upk ? nc : ~nc;  // true index; wraps to ~0 below 0
          const uint32_t rs = mx ? 1u : (my ? v.R : v.R * v.R);
          sib = ncr >= v.R ? CVX_NONE : (upk ? I + rs : I - rs);
        }
        const uint32_t link = mx ? rr.y : (my ? rr.z : rr.w);
        return (root || inner) ? sib : link;
      };
      // the canvas boundary has null links (CVX_NONE >= n_nodes) and so would
      // a broken pool (the two are told apart after the loop); a null
      // neighbour's load reads node 0 instead
      uint32_t Nn = neighbour(r);
      uint32_t In = Nn < v.n_nodes ? Nn : 0u;
      uint4 rn = ld_rec_t<SMALL>(rec, In);
      const float emin = mx ? eb.x : (my ? eb.y : eb.z);
      // certified when the lower bounds S_k - eb_k of the two other planes
      // exceed the upper bound Smin + emin of the minimum: each of the two
      // FP32 roundings is at most 2^-24 G of its plane, inside the 2^-23 G
      // each bound carries for it.  The minimum's own test is always false
      // (Smin - emin <= Smin + emin), so this is the majority of the three
      // (lane masks: scalar logic, no vector count)
      const float up_min = Smin + emin;
      const uint64_t s0 = lanes(S.x - eb.x > up_min);
      const uint64_t s1 = lanes(S.y - eb.y > up_min);
      const uint64_t s2 = lanes(S.z - eb.z > up_min);
      const bool cert = lane((s0 & s1) | (s2 & (s0 | s1)));
      // exit plane value and bound (the smallest one unless FP64 decides)
      float Sx = Smin, ex = emin;
      if (!cert) {
        // FP64 decision from the exact face planes, t = (X - o_k) / d_k with
        // the ray's reciprocal direction (as the FP64 caster does; an ulp or
        // two changes a decision only inside the 1e-12 face band)
        const double hd = ldexp(1.0, -(int)dep);
        double best = __builtin_inf();
        int kb = __builtin_ctz(kbit);
#pragma unroll 1
        for (int k = 0; k < 3; ++k) {
          const double X = (double)(get(c, k) ^ (get(up, k) ? 0u : ~0u)) * hd +
                           (get(up, k) ? hd : 0.0);
          const double tt = get(tD, k) == 0.0f ? __builtin_inf() : (X - slot.at(k)) * slot.at(6 + k);
          kb = tt < best ? k : kb;
          best = tt < best ? tt : best;
        }
        kbit = 1u << kb;
        mx = kb == 0;
        my = kb == 1;
        Sx = get(S, kb);
        ex = get(eb, kb);
        Nn = neighbour(ld_rec_t<SMALL>(rec, I));
        In = Nn < v.n_nodes ? Nn : 0u;
        rn = ld_rec_t<SMALL>(rec, In);
        need64 = true;
        out.flags |= CVX_RAYFLAG_FP64_EXIT;
        if (STATS) acc.fp64_exit++;
      }
      if (TRACE) {
        const double t = te_last + ldexp((double)Sx, -(int)db);
        for (int k = 0; k < 3; ++k) out.end[k] = slot.at(k) + t * slot.at(3 + k);
      }
      // SPLIT: does the piece end inside this leaf?  Certainly when the exit
      // lies beyond the end by more than both bounds, certainly not when it
      // lies before it by as much; otherwise the exit plane's exact FP64
      // parameter decides (an exit exactly at the end belongs to this piece,
      // and the next piece starts in the next leaf)
      bool cut = false;
      float Sl = Sx;  // where this leaf's segment ends
      if constexpr (SPLIT) {
        const float eb_end = ex + e_end;
        if (Sx + eb_end >= s_end) {
          if (Sx - eb_end > s_end) {
            cut = true;
          } else {
            const double hd = ldexp(1.0, -(int)dep);
            const int kx = __builtin_ctz(kbit);
            const double X = (double)(get(c, kx) ^ (get(up, kx) ? 0u : ~0u)) * hd +
                             (get(up, kx) ? hd : 0.0);
            cut = (X - slot.at(kx)) * slot.at(6 + kx) > t_end;
          }
        }
        Sl = cut ? s_end : Sx;
      }
      // length precision guard: rebase once the bound on this segment's
      // length exceeds 2^-10 of the leaf edge (w = 2^(db - dep) base cells),
      // compared in leaf edges (a power-of-two scale: exact)
      const float eseg = ex + e_ent;
      need64 = need64 || ldexpf(eseg, (int)dep - (int)db) > 0x1p-10f;
      float len = ldexpf(Sl - s_ent, (int)dep - (int)db);
      len = len > 0.0f ? len : 0.0f;
      // composite; every visited leaf is recorded: for a ray outside the face
      // band the exact segment is positive even when it rounds to 0 here
      // (kappa len as an FMA with a zero addend: the same rounding as the
      // product, with the FP16 kappa taken as an operand, no conversion)
      // (the absorbed share a = T - T e as one FMA, T updated in place)
      const float e =
          __builtin_amdgcn_exp2f(__builtin_fmaf(kappa_of(pay), len, 0.0f) * -1.4426950408889634f);
      const float a = __builtin_fmaf(-T, e, T);
      T = T * e;
      C.x = __builtin_fmaf(a, (float)(pay.x & 0xffu), C.x);
      C.y = __builtin_fmaf(a, (float)((pay.x >> 8) & 0xffu), C.y);
      C.z = __builtin_fmaf(a, (float)((pay.x >> 16) & 0xffu), C.z);
      if (TRACE) record(sk, n_rec, I, len);
      ++n_rec;
      if constexpr (SPLIT) {
        if (cut) break;  // the piece ends inside this leaf (no move, no flags)
      }
      // keeps the move (the first reader of the neighbour's record) after the
      // composite, so the record load has the whole step to arrive
      __builtin_amdgcn_sched_barrier(0);
      // ---- move to the neighbour (stop: bitwise, lane masks, not a branch)
      const bool mz = !mx & !my;
      const bool stop = (Nn >= v.n_nodes) | (use_stop & (T <= v.t_stop));
      if (stop) {
        end_Nn = Nn;
        end_nc = upk ? nc : ~nc;  // true index
        end_dep = dep;
        if constexpr (REFILL) {
          finish();
          write_pixel();
          alive = false;
          continue;
        }
        done = true;
      }
      // a ray that stopped still runs the move below (its results are not
      // used), on node 0 when its neighbour is null
      if (STATS) acc.outer += !inner && !stop;
      I = In;
      r = rn;
      pay = ld_pay_t<SMALL>(payp, I);
      const V3<uint32_t> co = c;
      c.x = mx ? nc : c.x;
      c.y = my ? nc : c.y;
      c.z = mz ? nc : c.z;
      s_ent = Sx;
      e_ent = ex;
      kbe = kbit;
      // far planes move by one cell on the exit axis, and for a coarser
      // leaf (m levels up) by the integer number of cells to its far planes:
      // in normalised indices the coarse cell's far plane lies after fine
      // cell (new | mask), so the plane advances by (new | mask) - old cells
      const uint32_t dL = (r.x & 1u) ? ((r.x >> 1) & 63u) : dep;
      const uint32_t m = dL < dep ? dep - dL : 0u;
      const uint32_t mask = (1u << m) - 1u;
      const uint32_t lw = db - dep;  // w = 2^lw
      for (int k = 0; k < 3; ++k) {
        const uint32_t cn = get(c, k);
        set(Nk, k, get(Nk, k) + (int32_t)(((cn | mask) - get(co, k)) << lw));
        set(c, k, (uint32_t)((int32_t)cn >> m));
      }
      w <<= m;
      dep -= m;
    }
    if (need64 && !done) {
      // FP64 rebase at the near face (axis bit kbe) of the current cell
      const int kr = kbe == 0u ? 0 : __builtin_ctz(kbe);
      const uint32_t cr = get(c, kr) ^ (get(up, kr) ? 0u : ~0u);  // true index
      const double Xp = (double)(get(up, kr) ? cr : cr + 1u) * ldexp(1.0, -(int)dep);
      const double te = (Xp - slot.at(kr)) * slot.at(6 + kr);
      for (int k = 0; k < 3; ++k) set(q, k, k == kr ? Xp : slot.at(k) + te * slot.at(3 + k));
      rebase(te);
    }
  }
  if constexpr (!REFILL) {
    finish();
    return;
  } else {
    const uint64_t waiting = __ballot(!alive);
    const uint32_t n_wait = (uint32_t)__popcll(waiting);
    if (next >= job->n_rays) {
      if (n_wait == 64u) return;
      wait_for = 64;  // no ray left: finish the ones in flight
      continue;
    }
    if (!alive) {
      const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
          (uint32_t)(waiting >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)waiting, 0u));
      if (next + rank < job->n_rays) alive = begin_job_ray(next + rank);
    }
    next += n_wait;
  }
  }
}

// ----------------------------------------------------------------------------
// FP64_PLAIN: canvas-global FP64; exit parameters from the exact face planes
// ((integer + side) 2^-dep - o_k) / d_k every step, FP64 compositing.
// ----------------------------------------------------------------------------
template <bool TRACE, bool STATS>
__device__ void cast_fp64(const DView& v, const V3<double>& d, const V3<double>& inv,
                          const Entry& en, const V3<bool>& up, Sink sk, Acc& acc, Out& out) {
  const V3<double> o{v.o[0], v.o[1], v.o[2]};
  const double Rd = (double)v.R;
  const void* rec = v.rec;
  const bool use_stop = v.alpha_stop < 1.0f;
  V3<double> q;
  for (int k = 0; k < 3; ++k) {
    double qk = get(o, k) + en.t0 * get(d, k);
    if (k == en.kin) qk = en.side ? Rd : 0.0;
    set(q, k, qk < 0.0 ? 0.0 : (qk > Rd ? Rd : qk));
  }
  uint32_t I, dep = 0;
  V3<uint32_t> c;
  uint4 r;
  const V3<uint32_t> C0 = deep_coords(q, up, v.R, v.max_depth);
  start_leaf(v, q, up, I, dep, c, r);
  bool bad = !descend_int(rec, v.n_nodes, C0, v.max_depth, I, dep, c, r);
  if (STATS) acc.descent += dep;
  double T = 1.0;
  V3<double> C{0.0, 0.0, 0.0};
  double t_ent = en.t0;
  uint32_t n_rec = 0;
  uint32_t step = 0;
  for (;; ++step) {
    if (step >= v.max_steps) { out.flags |= CVX_RAYFLAG_STEP_CAP; break; }
    if (bad) { out.flags |= CVX_RAYFLAG_BAD_LINK; break; }
    const double h = ldexp(1.0, -(int)dep);
    double best = __builtin_inf();
    int kx = 0;
    for (int k = 0; k < 3; ++k) {
      const double X = (double)(get(c, k) + (get(up, k) ? 1u : 0u)) * h;
      const double tt = get(d, k) == 0.0 ? __builtin_inf() : (X - get(o, k)) * get(inv, k);
      kx = tt < best ? k : kx;
      best = tt < best ? tt : best;
    }
    double len = ldexp(best - t_ent, (int)dep);
    len = len > 0.0 ? len : 0.0;
    if (TRACE)
      for (int k = 0; k < 3; ++k) out.end[k] = get(o, k) + best * get(d, k);
    double cr, cg, cb, kap;
    if (v.fmt == CVX_LEAF_F64) {
      const double4 p = ((const double4*)v.pay)[I];
      cr = p.x; cg = p.y; cb = p.z; kap = p.w;
    } else {
      const uint2 p = ((const uint2*)v.pay)[I];
      cr = (double)(p.x & 0xffu) / 255.0;
      cg = (double)((p.x >> 8) & 0xffu) / 255.0;
      cb = (double)((p.x >> 16) & 0xffu) / 255.0;
      kap = (double)kappa_of(p);
    }
    const double Tn = T * exp(-kap * len);
    const double a = T - Tn;
    C.x = __builtin_fma(a, cr, C.x);
    C.y = __builtin_fma(a, cg, C.y);
    C.z = __builtin_fma(a, cb, C.z);
    T = Tn;
    if (TRACE) record(sk, n_rec, I, len);
    ++n_rec;
    const uint32_t ck = get(c, kx);
    const bool upk = get(up, kx);
    const Move mv = neighbour(v, I, r, dep, ck, upk, kx);
    if (mv.at_edge || mv.N >= v.n_nodes || (use_stop && 1.0 - T >= (double)v.alpha_stop)) {
      if (!mv.at_edge && mv.N >= v.n_nodes) out.flags |= CVX_RAYFLAG_BAD_LINK;
      break;
    }
    if (STATS) acc.outer += mv.outer;
    const double X = (double)(upk ? mv.nc : ck) * h;
    set(c, kx, mv.nc);
    I = mv.N;
    r = ld_rec(rec, I);
    if (r.x & 1u) {
      const uint32_t dL = (r.x >> 1) & 63u;
      const uint32_t m = dL < dep ? dep - dL : 0u;
      for (int k = 0; k < 3; ++k) set(c, k, get(c, k) >> m);
      dep -= m;
    } else {
      for (int k = 0; k < 3; ++k) set(q, k, k == kx ? X : get(o, k) + best * get(d, k));
      const uint32_t d0 = dep;
      bad = !descend<double>(rec, v.n_nodes, q, up, I, dep, c, r);
      if (STATS) acc.descent += dep - d0;
    }
    t_ent = best > t_ent ? best : t_ent;
  }
  out.rgba[0] = C.x;
  out.rgba[1] = C.y;
  out.rgba[2] = C.z;
  out.rgba[3] = 1.0 - T;
  out.n = n_rec;
  out.steps = step + 1;
  if (STATS) acc.leaves += n_rec;
}

// ----------------------------------------------------------------------------
// FP32_NAIVE: canvas-global FP32 planes and points (drifts at depth).
// ----------------------------------------------------------------------------
template <bool TRACE, bool STATS>
__device__ void cast_naive(const DView& v, const V3<double>& d, const Entry& en, const V3<bool>& up,
                           Sink sk, Acc& acc, Out& out) {
  const void* rec = v.rec;
  const void* payp = v.pay;
  const bool use_stop = v.alpha_stop < 1.0f;
  V3<float> of, df, idf;
  for (int k = 0; k < 3; ++k) {
    set(of, k, (float)v.o[k]);
    set(df, k, (float)get(d, k));
    set(idf, k, get(df, k) == 0.0f ? 0.0f : 1.0f / get(df, k));
  }
  float t_ent = (float)en.t0;
  V3<float> q;
  for (int k = 0; k < 3; ++k)
    set(q, k, k == en.kin ? (en.side ? (float)v.R : 0.0f) : get(of, k) + t_ent * get(df, k));
  uint32_t I, dep = 0;
  V3<uint32_t> c;
  root_of<float>(q, up, v.R, c, I);
  uint4 r = ld_rec(rec, I);
  bool bad = !descend<float>(rec, v.n_nodes, q, up, I, dep, c, r);
  if (STATS) acc.descent += dep;
  float T = 1.0f;
  V3<float> C{0.f, 0.f, 0.f};
  uint32_t n_rec = 0;
  uint32_t step = 0;
  for (;; ++step) {
    if (step >= v.max_steps) { out.flags |= CVX_RAYFLAG_STEP_CAP; break; }
    if (bad) { out.flags |= CVX_RAYFLAG_BAD_LINK; break; }
    const float h = ldexpf(1.0f, -(int)dep);
    float best = BIGF, Xb = 0.0f;
    int kx = 0;
    for (int k = 0; k < 3; ++k) {
      const float X = (float)(get(c, k) + (get(up, k) ? 1u : 0u)) * h;
      const float tt = get(df, k) == 0.0f ? BIGF : (X - get(of, k)) * get(idf, k);
      kx = tt < best ? k : kx;
      Xb = tt < best ? X : Xb;
      best = tt < best ? tt : best;
    }
    float len = (best - t_ent) * ldexpf(1.0f, (int)dep);
    len = len > 0.0f ? len : 0.0f;
    if (TRACE)
      for (int k = 0; k < 3; ++k)
        out.end[k] = k == kx ? (double)Xb : (double)(get(of, k) + best * get(df, k));
    const uint2 pay = ld_pay(payp, I);
    const float Tn = T * __builtin_amdgcn_exp2f(kappa_of(pay) * len * -1.4426950408889634f);
    const float a = T - Tn;
    C.x = __builtin_fmaf(a, (float)(pay.x & 0xffu), C.x);
    C.y = __builtin_fmaf(a, (float)((pay.x >> 8) & 0xffu), C.y);
    C.z = __builtin_fmaf(a, (float)((pay.x >> 16) & 0xffu), C.z);
    T = Tn;
    if (TRACE) record(sk, n_rec, I, len);
    ++n_rec;
    const uint32_t ck = get(c, kx);
    const bool upk = get(up, kx);
    const Move mv = neighbour(v, I, r, dep, ck, upk, kx);
    if (mv.at_edge || mv.N >= v.n_nodes || (use_stop && 1.0f - T >= v.alpha_stop)) {
      if (!mv.at_edge && mv.N >= v.n_nodes) out.flags |= CVX_RAYFLAG_BAD_LINK;
      break;
    }
    if (STATS) acc.outer += mv.outer;
    set(c, kx, mv.nc);
    I = mv.N;
    r = ld_rec(rec, I);
    if (r.x & 1u) {
      const uint32_t dL = (r.x >> 1) & 63u;
      const uint32_t m = dL < dep ? dep - dL : 0u;
      for (int k = 0; k < 3; ++k) set(c, k, get(c, k) >> m);
      dep -= m;
    } else {
      for (int k = 0; k < 3; ++k) set(q, k, k == kx ? Xb : get(of, k) + best * get(df, k));
      const uint32_t d0 = dep;
      bad = !descend<float>(rec, v.n_nodes, q, up, I, dep, c, r);
      if (STATS) acc.descent += dep - d0;
    }
    t_ent = best > t_ent ? best : t_ent;
  }
  const float k255 = 1.0f / 255.0f;
  out.rgba[0] = C.x * k255;
  out.rgba[1] = C.y * k255;
  out.rgba[2] = C.z * k255;
  out.rgba[3] = 1.0f - T;
  out.n = n_rec;
  out.steps = step + 1;
  if (STATS) acc.leaves += n_rec;
}

// ----------------------------------------------------------------------------
// FP32_CELL_LOCAL / FP16_CELL_LOCAL: the paper's traversal (Sec. 6.2).  The
// entry point p of the current leaf is held in the leaf's own frame (origin at
// its centre, edge 1) in FP32 (or FP16); the exit face is the argmin of
// t_k = (+-0.5 - p_k) / d_k, the exit point p' = p + t d, and p' is mapped into
// the next cell by a power-of-two scale and a shift (across a face: shift by
// one edge on that axis; into a coarser leaf: scale by 2^-m after the integer
// offset of the finer cell; into a refined cell: child by the sign of p, then
// p -> 2p - b + 1/2 per level).  The start point is the only FP64 step
// (rounded once into the first leaf's frame).  Nothing is certified: this is
// the scheme whose error Sec. 6.3 bounds, measured by the precision
// experiment.  In FP16 every operation of the traversal (t, p', the frame
// changes, the ray direction itself) is rounded to half precision; a coarser
// leaf's frame change is p' s + c with s = 2^-m and c = (offset + 1/2) s - 1/2
// each rounded once to half.  Compositing stays in FP32 in both.
// ----------------------------------------------------------------------------
__device__ __forceinline__ float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ _Float16 fma_r(_Float16 a, _Float16 b, _Float16 c) {
  return __builtin_fmaf16(a, b, c);
}

template <class Real, bool TRACE, bool STATS>
__device__ void cast_local(const DView& v, const V3<double>& d, const Entry& en, const V3<bool>& up,
                           Sink sk, Acc& acc, Out& out) {
  constexpr bool HALF = __is_same(Real, _Float16);
  const Real inf = (Real)__builtin_inff();
  const V3<double> o{v.o[0], v.o[1], v.o[2]};
  const double Rd = (double)v.R;
  const void* rec = v.rec;
  const void* payp = v.pay;
  const bool use_stop = v.alpha_stop < 1.0f;
  const V3<Real> df{(Real)d.x, (Real)d.y, (Real)d.z};
  V3<double> q;
  for (int k = 0; k < 3; ++k) {
    double qk = get(o, k) + en.t0 * get(d, k);
    if (k == en.kin) qk = en.side ? Rd : 0.0;
    set(q, k, qk < 0.0 ? 0.0 : (qk > Rd ? Rd : qk));
  }
  uint32_t I, dep = 0;
  V3<uint32_t> c;
  uint4 r;
  const V3<uint32_t> C0 = deep_coords(q, up, v.R, v.max_depth);
  start_leaf(v, q, up, I, dep, c, r);
  bool bad = !descend_int(rec, v.n_nodes, C0, v.max_depth, I, dep, c, r);
  if (STATS) acc.descent += dep;
  V3<Real> p;
  for (int k = 0; k < 3; ++k)
    set(p, k, (Real)(ldexp(get(q, k), (int)dep) - (double)get(c, k) - 0.5));
  float T = 1.0f;
  V3<float> C{0.f, 0.f, 0.f};
  uint32_t n_rec = 0;
  uint32_t step = 0;
  for (;; ++step) {
    if (step >= v.max_steps) { out.flags |= CVX_RAYFLAG_STEP_CAP; break; }
    if (bad) { out.flags |= CVX_RAYFLAG_BAD_LINK; break; }
    Real best = HALF ? inf : (Real)BIGF;
    int kx = 0;
    for (int k = 0; k < 3; ++k) {
      const Real face = get(up, k) ? (Real)0.5f : (Real)-0.5f;
      const Real tt = get(df, k) == (Real)0.0f ? (HALF ? inf : (Real)BIGF)
                                                : (face - get(p, k)) / get(df, k);
      kx = tt < best ? k : kx;
      best = tt < best ? tt : best;
    }
    const Real len = best > (Real)0.0f ? best : (Real)0.0f;   // leaf edges
    V3<Real> pe;
    for (int k = 0; k < 3; ++k) set(pe, k, fma_r(len, get(df, k), get(p, k)));
    if (TRACE) {
      const double h = ldexp(1.0, -(int)dep);
      for (int k = 0; k < 3; ++k)
        out.end[k] = ((double)get(c, k) + 0.5 + (double)get(pe, k)) * h;
    }
    const uint2 pay = ld_pay(payp, I);
    const float lenf = (float)len;
    const float Tn = T * __builtin_amdgcn_exp2f(kappa_of(pay) * lenf * -1.4426950408889634f);
    const float a = T - Tn;
    C.x = __builtin_fmaf(a, (float)(pay.x & 0xffu), C.x);
    C.y = __builtin_fmaf(a, (float)((pay.x >> 8) & 0xffu), C.y);
    C.z = __builtin_fmaf(a, (float)((pay.x >> 16) & 0xffu), C.z);
    T = Tn;
    if (TRACE) record(sk, n_rec, I, lenf);
    ++n_rec;
    const uint32_t ck = get(c, kx);
    const bool upk = get(up, kx);
    const Move mv = neighbour(v, I, r, dep, ck, upk, kx);
    if (mv.at_edge || mv.N >= v.n_nodes || (use_stop && 1.0f - T >= v.alpha_stop)) {
      if (!mv.at_edge && mv.N >= v.n_nodes) out.flags |= CVX_RAYFLAG_BAD_LINK;
      break;
    }
    if (STATS) acc.outer += mv.outer;
    // across the face: one edge along kx
    p = pe;
    set(p, kx, get(pe, kx) - (upk ? (Real)1.0f : (Real)-1.0f));
    set(c, kx, mv.nc);
    I = mv.N;
    r = ld_rec(rec, I);
    if (r.x & 1u) {
      // a coarser leaf: scale by 2^-m after the offset of the finer cell in it
      const uint32_t dL = (r.x >> 1) & 63u;
      const uint32_t m = dL < dep ? dep - dL : 0u;
      const float sc = ldexpf(1.0f, -(int)m);
      const uint32_t mask = (1u << m) - 1u;
      for (int k = 0; k < 3; ++k) {
        const float off = (float)(get(c, k) & mask);
        if constexpr (HALF)
          set(p, k, fma_r(get(p, k), (Real)sc, (Real)__builtin_fmaf(off + 0.5f, sc, -0.5f)));
        else
          set(p, k, __builtin_fmaf(get(p, k) + 0.5f + off, sc, -0.5f));
        set(c, k, get(c, k) >> m);
      }
      dep -= m;
    } else {
      // a refined cell: children by the sign of p, ties to the side the ray moves into
      const uint32_t d0 = dep;
      while (!(r.x & 1u)) {
        if (r.x >= v.n_nodes - 7u) { bad = true; break; }
        uint32_t oct = 0;
        for (int k = 0; k < 3; ++k) {
          const Real pk = get(p, k);
          const uint32_t b = (pk > (Real)0.0f || (pk == (Real)0.0f && get(up, k))) ? 1u : 0u;
          oct |= b << k;
          set(p, k, (Real)2.0f * pk - (Real)(float)b + (Real)0.5f);
          set(c, k, 2u * get(c, k) + b);
        }
        I = r.x + oct;
        ++dep;
        r = ld_rec(rec, I);
      }
      if (STATS) acc.descent += dep - d0;
    }
  }
  const float k255 = 1.0f / 255.0f;
  out.rgba[0] = C.x * k255;
  out.rgba[1] = C.y * k255;
  out.rgba[2] = C.z * k255;
  out.rgba[3] = 1.0f - T;
  out.n = n_rec;
  out.steps = step + 1;
  if (STATS) acc.leaves += n_rec;
}

// One ray, or with SPLIT its chord piece `piece` of `pieces`: the canvas
// chord [t0, t1] cut at t0 + (t1 - t0) f_j, f_j = (67 j + 1) / (67 pieces)
// (the same FP64 expression for the end of piece j - 1 and the start of
// piece j).  A cut at j / pieces would fall exactly on a cell plane whenever
// the chord runs between opposite canvas faces of one axis (the midpoint of
// [0, R] is a plane), where the end test of one piece and the point location
// of the next could round to different sides; with the factor 67 (no root
// array side has it) the cut points are not dyadic.
template <int VAR, bool TRACE, bool STATS, bool SMALL = false, bool SPLIT = false>
__device__ void cast_ray(const DView& v, uint32_t px, uint32_t py, Sink sk, Acc& acc, Out& out,
                         uint32_t piece = 0, uint32_t pieces = 1) {
  const RaySlot slot{(lds_f64*)(s_ray + threadIdx.x), blockDim.x};
  const V3<double> d = ray_dir(v, px, py);
  const V3<double> o{v.o[0], v.o[1], v.o[2]};
  out.rgba[0] = out.rgba[1] = out.rgba[2] = out.rgba[3] = 0.0;
  out.T = 1.0;
  out.flags = 0;
  out.n = 0;
  out.steps = 0;
  out.end[0] = out.end[1] = out.end[2] = 0.0;
  if (STATS) acc.rays++;
  const V3<double> inv{rcp_nr(d.x), rcp_nr(d.y), rcp_nr(d.z)};
  const Entry en = canvas_entry(o, d, inv, (double)v.R);
  if (!en.hit) return;
  const V3<bool> up{d.x > 0.0, d.y > 0.0, d.z > 0.0};
  if constexpr (SPLIT) {
    static_assert(VAR == (int)CVX_VARIANT_FP32_REBASED, "chord pieces: FP32_REBASED only");
    const double span = en.t1 - en.t0;
    const double den = 67.0 * (double)pieces;
    Entry ep = en;
    if (piece > 0) {  // starts inside the chord, on no face
      ep.t0 = en.t0 + span * (double)(67u * piece + 1u) / den;
      ep.kin = -1;
    }
    const double t_end = piece + 1 < pieces
                             ? en.t0 + span * (double)(67u * (piece + 1u) + 1u) / den
                             : __builtin_inf();
    cast_fp32<TRACE, STATS, SMALL, false, true>(v, slot, o, d, inv, ep, up, sk, acc, out, nullptr,
                                                t_end, piece == 0);
  } else if constexpr (VAR == (int)CVX_VARIANT_FP32_REBASED) {
    cast_fp32<TRACE, STATS, SMALL>(v, slot, o, d, inv, en, up, sk, acc, out);
  } else if constexpr (VAR == (int)CVX_VARIANT_FP64_PLAIN) {
    cast_fp64<TRACE, STATS>(v, d, inv, en, up, sk, acc, out);
  } else if constexpr (VAR == (int)CVX_VARIANT_FP32_NAIVE) {
    cast_naive<TRACE, STATS>(v, d, en, up, sk, acc, out);
  } else if constexpr (VAR == (int)CVX_VARIANT_FP32_CELL_LOCAL) {
    cast_local<float, TRACE, STATS>(v, d, en, up, sk, acc, out);
  } else {
    cast_local<_Float16, TRACE, STATS>(v, d, en, up, sk, acc, out);
  }
}

// View table reads through the constant address space: the table is
// read-only while the kernel runs, so at a uniform index (render mode: a
// tile never straddles views) the compiler issues scalar loads straight into
// scalar registers instead of vector loads and a readfirstlane per word.
typedef const __attribute__((address_space(4))) uint32_t cu32_t;
__device__ __forceinline__ DView view_const(const DView* views, int i) {
  const cu32_t* q = (const cu32_t*)(views + i);
  uint32_t w[sizeof(DView) / 4];
  for (int j = 0; j < (int)(sizeof(DView) / 4); ++j) w[j] = q[j];
  DView u;
  __builtin_memcpy(&u, w, sizeof(DView));
  return u;
}
__device__ __forceinline__ uint64_t view_first_tile(const DView* views, int i) {
  const cu32_t* q = (const cu32_t*)&views[i].first_tile;
  return (uint64_t)q[0] | ((uint64_t)q[1] << 32);
}

// Copy of a view that is the same in every lane (render mode: a tile never
// straddles views), read into scalar registers, so the pool pointers and
// sizes do not occupy vector registers during the traversal.
__device__ __forceinline__ DView uniform_view(const DView& v) {
  constexpr int n = sizeof(DView) / 4;
  uint32_t w[n];
  __builtin_memcpy(w, &v, sizeof(DView));
  for (int i = 0; i < n; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  DView u;
  __builtin_memcpy(&u, w, sizeof(DView));
  return u;
}

// SPLIT: every view with pieces > 1 has pieces work items per tile (tile
// t, piece j at t * pieces + j); each piece writes its colour and
// transmittance to a.split_tmp[pixel * a.pieces + j] for k_merge_pieces.  In
// trace mode the rows are (ray, piece) pairs, ray-major, a.pieces per ray.
template <int VAR, bool TRACE, bool STATS, bool OUT64, bool SMALL = false, bool SPLIT = false>
__device__ __forceinline__ void cast_grid(const CastArgs& a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t total = a.hdr->total_work;
  const uint32_t nv = a.hdr->n_views;
  Acc acc = {0, 0, 0, 0, 0, 0, 0, 0};
  const uint32_t nq = a.hdr->n_queues;  // 1 or CVX_NQ (a power of two)
  uint32_t qi = blockIdx.x & (nq - 1u), drained = 0;
  for (;;) {
    // next item of range qi; an exhausted range passes on to the next one
    const uint64_t q_lo = total * qi / nq, q_hi = total * (qi + 1u) / nq;
    uint32_t taken = 0;
    if (lane == 0) taken = atomicAdd(&a.hdr->queue[qi].next, 1u);
    // every lane is active here (the loop exit is uniform), so the first
    // active lane is lane 0
    taken = __builtin_amdgcn_readfirstlane(taken);
    if (q_lo + taken >= q_hi) {
      if (++drained == nq) break;
      qi = (qi + 1u) & (nq - 1u);
      continue;
    }
    const uint32_t w = (uint32_t)(q_lo + taken);
    Out res;
    res.steps = 0;
    if constexpr (!TRACE) {
      int lo = 0, hi = (int)nv - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (view_first_tile(a.views, mid) <= (uint64_t)w) lo = mid; else hi = mid - 1;
      }
      const DView v = view_const(a.views, lo);
      uint64_t t = (uint64_t)w - v.first_tile;
      uint32_t piece = 0;
      if constexpr (SPLIT) {
        piece = (uint32_t)(t % v.pieces);
        t /= v.pieces;
      }
      const uint32_t tx = (uint32_t)(t % v.tiles_x), ty = (uint32_t)(t / v.tiles_x);
      const uint32_t x = tx * a.tile_w + lane % a.tile_w, y = ty * a.tile_h + lane / a.tile_w;
      if (x < v.W && y < v.H) {
        Sink sk{nullptr, nullptr, nullptr, 0};
        cast_ray<VAR, false, STATS, SMALL, SPLIT>(v, x, y, sk, acc, res, piece, v.pieces);
        const uint64_t pix = v.out_off + (uint64_t)y * v.W + x;
        if (SPLIT && v.pieces > 1) {
          ((float4*)a.split_tmp)[pix * a.pieces + piece] =
              make_float4((float)res.rgba[0], (float)res.rgba[1], (float)res.rgba[2],
                          (float)res.T);
        } else if constexpr (OUT64) {
          double2* o2 = (double2*)a.out + 2 * pix;
          o2[0] = make_double2(res.rgba[0], res.rgba[1]);
          o2[1] = make_double2(res.rgba[2], res.rgba[3]);
        } else {
          ((float4*)a.out)[pix] = make_float4((float)res.rgba[0], (float)res.rgba[1],
                                              (float)res.rgba[2], (float)res.rgba[3]);
        }
      }
    } else {
      const uint64_t ri = (uint64_t)w * 64u + lane;
      if (ri < a.hdr->n_rays) {
        // SPLIT: row ri is piece ri % a.pieces of ray ri / a.pieces
        const uint64_t ray = SPLIT ? ri / a.pieces : ri;
        const uint32_t piece = SPLIT ? (uint32_t)(ri % a.pieces) : 0u;
        const uint64_t id = a.ray_ids[ray];
        const uint32_t vi = (uint32_t)(id >> 32), pix = (uint32_t)(id & 0xffffffffu);
        a.n_leaves[ri] = 0;
        a.flags[ri] = CVX_RAYFLAG_BAD_LINK;
        if (vi < nv) {
          const DView& v = a.views[vi];
          if ((uint64_t)pix < (uint64_t)v.W * v.H) {
            Sink sk{a.leaf_ids + ri * a.max_leaves,
                    a.local_len ? a.local_len + ri * a.max_leaves : nullptr,
                    a.local_len64 ? a.local_len64 + ri * a.max_leaves : nullptr, a.max_leaves};
            if (!SPLIT || piece < v.pieces) {
              cast_ray<VAR, TRACE, STATS, SMALL, SPLIT>(v, pix % v.W, pix / v.W, sk, acc, res,
                                                         piece, v.pieces);
            } else {  // an unsplit view: its rays have one piece, the others are empty
              res.rgba[0] = res.rgba[1] = res.rgba[2] = res.rgba[3] = 0.0;
              res.T = 1.0;
              res.flags = 0;
              res.n = 0;
              res.end[0] = res.end[1] = res.end[2] = 0.0;
            }
            a.n_leaves[ri] = res.n;
            a.flags[ri] = res.flags;
            if (a.end_point)
              for (int k = 0; k < 3; ++k) a.end_point[3 * ri + k] = res.end[k];
            // with pieces, a row holds its piece's colour and transmittance
            ((float4*)a.trace_rgba)[ri] =
                make_float4((float)res.rgba[0], (float)res.rgba[1], (float)res.rgba[2],
                            SPLIT ? (float)res.T : (float)res.rgba[3]);
          }
        }
      }
    }
    if constexpr (STATS) {
      // every lane of the wavefront is here: the tile took as many
      // iterations as its longest ray
      uint32_t m = res.steps;
      for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = __shfl_xor(m, off, 64);
        m = o > m ? o : m;
      }
      acc.steps += res.steps;
      acc.slots += m;
    }
  }
  if constexpr (STATS) {
    const uint64_t vals[8] = {acc.rays, acc.leaves, acc.outer, acc.descent,
                              acc.fp64_exit, acc.rebase, acc.steps, acc.slots};
    for (int s = 0; s < 8; ++s) {
      unsigned long long x = vals[s];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
      if (lane == 0 && x) atomicAdd((unsigned long long*)&a.stats[s], (unsigned long long)x);
    }
  }
}

// The FP32 render with lane refill: a work item is up to a.item_tiles
// consecutive tiles of one view (items never straddle views, so the view
// stays wavefront-uniform), whose rays the wavefront's lanes take in turn
// (RefillJob).  Per-view item counts replace tile counts in the views'
// prefix sums (first_tile) and in the header's total.
template <bool SMALL>
__device__ __forceinline__ void cast_grid_refill(const CastArgs& a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t total = a.hdr->total_work;
  const uint32_t nv = a.hdr->n_views;
  const uint32_t nq = a.hdr->n_queues;  // 1 or CVX_NQ (a power of two)
  const RaySlot slot{(lds_f64*)(s_ray + threadIdx.x), blockDim.x};
  uint32_t qi = blockIdx.x & (nq - 1u), drained = 0;
  for (;;) {
    const uint64_t q_lo = total * qi / nq, q_hi = total * (qi + 1u) / nq;
    uint32_t taken = 0;
    if (lane == 0) taken = atomicAdd(&a.hdr->queue[qi].next, 1u);
    taken = __builtin_amdgcn_readfirstlane(taken);
    if (q_lo + taken >= q_hi) {
      if (++drained == nq) break;
      qi = (qi + 1u) & (nq - 1u);
      continue;
    }
    const uint32_t w = (uint32_t)(q_lo + taken);
    int lo = 0, hi = (int)nv - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (a.views[mid].first_tile <= (uint64_t)w) lo = mid; else hi = mid - 1;
    }
    const DView v = uniform_view(a.views[lo]);
    const uint64_t tiles = (uint64_t)v.tiles_x * ((v.H + a.tile_h - 1u) / a.tile_h);
    RefillJob job;
    job.out = (float4*)a.out;
    job.first_tile = ((uint64_t)w - v.first_tile) * a.item_tiles;
    const uint64_t nt = tiles - job.first_tile < a.item_tiles ? tiles - job.first_tile : a.item_tiles;
    job.n_rays = (uint32_t)nt * 64u;
    job.tile_w = a.tile_w;
    job.tile_h = a.tile_h;
    job.refill_min = a.refill_min;
    Out res;
    Acc acc = {0, 0, 0, 0, 0, 0, 0, 0};
    Sink sk{nullptr, nullptr, nullptr, 0};
    const V3<double> z{0.0, 0.0, 0.0};
    const Entry en{0.0, 0.0, -1, 0, false};
    cast_fp32<false, false, SMALL, true>(v, slot, z, z, z, en, V3<bool>{false, false, false}, sk,
                                         acc, res, &job);
  }
}

template <int VAR, bool TRACE, bool STATS, bool OUT64, bool SPLIT = false>
__global__ __launch_bounds__(256) void k_cast(CastArgs a) {
  cast_grid<VAR, TRACE, STATS, OUT64, false, SPLIT>(a);
}

// Render-mode entry points with an occupancy target (trace and stats
// instances use k_cast).  The FP32 caster fits eight wavefronts per SIMD
// without spills (its LDS slot, 72 B per lane, then fills 147 KB of a CU's
// 160 KB).
template <bool OUT64, bool SMALL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CVX_CAST32_WAVES))) void k_cast32(
    CastArgs a) {
  cast_grid<(int)CVX_VARIANT_FP32_REBASED, false, false, OUT64, SMALL>(a);
}

// The FP32 render of chord pieces (views with pieces > 1; the others as
// k_cast32), with the same occupancy target.
template <bool SMALL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CVX_CAST32_WAVES))) void k_cast32s(
    CastArgs a) {
  cast_grid<(int)CVX_VARIANT_FP32_REBASED, false, false, false, SMALL, true>(a);
}

// Front-to-back merge of the chord pieces of every pixel of the split views
// (blockIdx.y = view): C = C_0 + T_0 C_1 + T_0 T_1 C_2 + ..., the pixel's
// alpha 1 - T_0 T_1 ...  (the associative over operator on (C, T) pairs).
__global__ void k_merge_pieces(const DView* views, const CastHeader* hdr, const float4* tmp,
                               float4* out, uint32_t stride) {
  if (blockIdx.y >= hdr->n_views) return;  // the count of this call (graphs replay)
  const DView& v = views[blockIdx.y];
  if (v.pieces <= 1u) return;
  const uint64_t n = (uint64_t)v.W * v.H;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t pix = v.out_off + i;
    float cr = 0.0f, cg = 0.0f, cb = 0.0f, T = 1.0f;
    for (uint32_t j = 0; j < v.pieces; ++j) {
      const float4 q = tmp[pix * stride + j];
      cr = __builtin_fmaf(T, q.x, cr);
      cg = __builtin_fmaf(T, q.y, cg);
      cb = __builtin_fmaf(T, q.z, cb);
      T *= q.w;
    }
    out[pix] = make_float4(cr, cg, cb, 1.0f - T);
  }
}

// The refilling render keeps the ray setup inside its loop; seven
// wavefronts per SIMD leave it the registers to do so without spills.
template <bool SMALL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CVX_CAST32R_WAVES))) void k_cast32r(
    CastArgs a) {
  cast_grid_refill<SMALL>(a);
}

// The FP64 caster keeps its direction, reciprocal and eye in registers (they
// enter every step); seven wavefronts per SIMD fit without spills.
template <bool TRACE, bool STATS, bool OUT64>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7))) void k_cast64(
    CastArgs a) {
  cast_grid<(int)CVX_VARIANT_FP64_PLAIN, TRACE, STATS, OUT64>(a);
}

// One thread per view: the leaf holding the eye, when every ray of the view
// starts there (eye strictly inside the canvas and off every plane of the
// deepest grid: the slab test then gives t0 = 0 and the start point is the
// eye itself for every direction).  The first CVX_NQ threads also clear the
// work-queue heads (the staged header arrives with them at zero; a cleared
// head keeps a replayed launch safe on its own).
__global__ void k_view_starts(DView* views, CastHeader* hdr, uint32_t enable) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < CVX_NQ) hdr->queue[i].next = 0u;
  if (i >= hdr->n_views) return;  // the count of this call (a graph replays the launch)
  DView& v = views[i];
  v.start_ok = 0u;
  if (!enable) return;
  const double Rd = (double)v.R;
  bool ok = true;
  for (int k = 0; k < 3; ++k) {
    const double Q = ldexp(v.o[k], (int)v.max_depth);
    ok = ok && v.o[k] > 0.0 && v.o[k] < Rd && floor(Q) != Q;
  }
  if (!ok) return;
  const V3<double> q{v.o[0], v.o[1], v.o[2]};
  const V3<bool> up{true, true, true};  // no plane ties: the direction plays no part
  const V3<uint32_t> C = deep_coords(q, up, v.R, v.max_depth);
  uint32_t I, dep;
  V3<uint32_t> c;
  uint4 r;
  locate_top(v, C, I, dep, c, r);
  if (!descend_int(v.rec, v.n_nodes, C, v.max_depth, I, dep, c, r)) return;
  v.start_node = I;
  v.start_dep = dep;
  v.start_c[0] = c.x;
  v.start_c[1] = c.y;
  v.start_c[2] = c.z;
  v.start_ok = 1u;
}

template <int VAR, bool TRACE, bool STATS, bool OUT64>
int launch_t(void* stream, const CastArgs& a, uint32_t wgs, uint32_t wg_size) {
  const size_t lds = VAR == (int)CVX_VARIANT_FP32_REBASED ? 9u * sizeof(double) * wg_size : 0u;
  if constexpr (VAR == (int)CVX_VARIANT_FP64_PLAIN && !TRACE && !STATS)
    hipLaunchKernelGGL((k_cast64<TRACE, STATS, OUT64>), dim3(wgs), dim3(wg_size), lds,
                       (hipStream_t)stream, a);
  else if constexpr (VAR == (int)CVX_VARIANT_FP32_REBASED && TRACE && !STATS && !OUT64) {
    if (a.pieces > 1u)
      hipLaunchKernelGGL((k_cast<VAR, true, false, false, true>), dim3(wgs), dim3(wg_size), lds,
                         (hipStream_t)stream, a);
    else
      hipLaunchKernelGGL((k_cast<VAR, true, false, false>), dim3(wgs), dim3(wg_size), lds,
                         (hipStream_t)stream, a);
  } else if constexpr (VAR == (int)CVX_VARIANT_FP32_REBASED && !TRACE && !STATS && !OUT64) {
    if (a.pieces > 1u) {
      if (a.small_pools)
        hipLaunchKernelGGL((k_cast32s<true>), dim3(wgs), dim3(wg_size), lds, (hipStream_t)stream,
                           a);
      else
        hipLaunchKernelGGL((k_cast32s<false>), dim3(wgs), dim3(wg_size), lds, (hipStream_t)stream,
                           a);
    } else if (a.item_tiles > 1u) {
      if (a.small_pools)
        hipLaunchKernelGGL((k_cast32r<true>), dim3(wgs), dim3(wg_size), lds, (hipStream_t)stream,
                           a);
      else
        hipLaunchKernelGGL((k_cast32r<false>), dim3(wgs), dim3(wg_size), lds, (hipStream_t)stream,
                           a);
    } else if (a.small_pools) {
      hipLaunchKernelGGL((k_cast32<OUT64, true>), dim3(wgs), dim3(wg_size), lds,
                         (hipStream_t)stream, a);
    } else {
      hipLaunchKernelGGL((k_cast32<OUT64, false>), dim3(wgs), dim3(wg_size), lds,
                         (hipStream_t)stream, a);
    }
  }
  else
    hipLaunchKernelGGL((k_cast<VAR, TRACE, STATS, OUT64>), dim3(wgs), dim3(wg_size), lds,
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
    case CVX_VARIANT_FP32_CELL_LOCAL:
      return launch_v<(int)CVX_VARIANT_FP32_CELL_LOCAL>(stream, trace, stats, false, a,
                                                        workgroups, wg_size);
    case CVX_VARIANT_FP16_CELL_LOCAL:
      return launch_v<(int)CVX_VARIANT_FP16_CELL_LOCAL>(stream, trace, stats, false, a,
                                                        workgroups, wg_size);
    default:
      return (int)hipErrorInvalidValue;
  }
}

int launch_view_starts(void* stream, DView* views, CastHeader* hdr, uint32_t enable) {
  hipLaunchKernelGGL(k_view_starts, dim3((CVX_MAX_VIEWS + 63u) / 64u), dim3(64), 0,
                     (hipStream_t)stream, views, hdr, enable);
  return (int)hipGetLastError();
}

int launch_merge_pieces(void* stream, const DView* views, const CastHeader* hdr, uint32_t n_views,
                        const void* tmp, void* out, uint32_t stride) {
  hipLaunchKernelGGL(k_merge_pieces, dim3(256, n_views), dim3(256), 0, (hipStream_t)stream, views,
                     hdr, (const float4*)tmp, (float4*)out, stride);
  return (int)hipGetLastError();
}

// Device memory of cvx_render_noalloc: the call's CastHeader, then its view
// table (CVX_NOALLOC_MAX_VIEWS records).  Each GPU holds its own copy for
// the life of the process.  Host code never passes this name to a kernel or
// a copy: the address on a device comes from scratch_address.
static __device__ __align__(256) unsigned char scratch[CVX_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;

int scratch_address(int device, void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxScratchDevices] = {};
  if (device < 0 || device >= kMaxScratchDevices) return (int)hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    if (!p) return (int)hipErrorInvalidSymbol;
    addr[device] = p;
  }
  *ptr = addr[device];
  return (int)hipSuccess;
}

}  // namespace cvx

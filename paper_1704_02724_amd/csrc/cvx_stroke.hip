// Painting a brush stroke into a resident pool (Sec. 5.1-5.3).
//
// A stroke is a list of spherical stamps with one brush colour, one opacity
// density per brush radius and one brush radius.  Its full effect on a leaf:
// a leaf the stamps overlap is split while its edge exceeds radius / k and it
// is above the canvas max depth (Sec. 5.2; the children inherit its colour and
// half its optical depth per edge); a leaf that is not split and whose centre
// lies in a stamp takes the stroke once with the additive density mix of
// Sec. 5.1.  Sec. 5.3 defers the splits: the stroke is first painted into the
// leaves that exist (immediate feedback), then the tree is refined one level
// per frame.
//
// k_stroke_visit does one level of that walk for a frontier of cells, one
// thread per cell: cells the stamps miss are left alone; refined cells push
// their 8 children to the next frontier; a leaf that still needs a split is
// appended to the pending list with its payload as it was before the stroke
// (its children must inherit that, not the immediate paint); a leaf whose
// centre lies in a stamp is painted in place.  In merge mode (a coarsening
// stroke, once its splits are done) the walk lists the refined cells the
// stamps overlap whose 8 children are leaves with identical payload bytes,
// and paints nothing.  Box and centre tests and the
// mix are FP64 with the operations in the order of their definition
// (no contraction), so the result does not depend on the launch.
#include <hip/hip_runtime.h>

#include "cvx_internal.h"

namespace cvx {

namespace {

__device__ __forceinline__ double box_dist2(const double lo[3], double e, const double4 s) {
  const double sc[3] = {s.x, s.y, s.z};
  double d2 = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double v = fmax(fmax(lo[k] - sc[k], 0.0), sc[k] - (lo[k] + e));
    d2 += v * v;
  }
  return d2;
}

__device__ __forceinline__ double centre_dist2(const double lo[3], double e, const double4 s) {
  const double cx = lo[0] + 0.5 * e - s.x;
  const double cy = lo[1] + 0.5 * e - s.y;
  const double cz = lo[2] + 0.5 * e - s.z;
  return cx * cx + cy * cy + cz * cz;
}

__device__ __forceinline__ uint32_t to_byte(double v) {
  return (uint32_t)rint(255.0 * fmin(fmax(v, 0.0), 1.0));
}

// Additive density mix of one stroke into a leaf of edge e (Sec. 5.1, density
// read as the alpha term): kb = sigma e / radius, m = kb / (kb + kappa).
__device__ void paint_leaf(void* pay, uint32_t node, uint32_t fmt, double e,
                           const StrokeArgs& a) {
  double q[4];
  if (fmt == CVX_LEAF_F64) {
    const double* p = (const double*)pay + 4 * (uint64_t)node;
    for (int c = 0; c < 4; ++c) q[c] = p[c];
  } else {
    const uint2 p = ((const uint2*)pay)[node];
    q[0] = (double)(p.x & 0xffu) / 255.0;
    q[1] = (double)((p.x >> 8) & 0xffu) / 255.0;
    q[2] = (double)((p.x >> 16) & 0xffu) / 255.0;
    q[3] = (double)__builtin_bit_cast(_Float16, (unsigned short)(p.y & 0xffffu));
  }
  const double kb = a.sigma * e / a.radius;
  const double kc = q[3];
  const double m = (kb + kc) > 0.0 ? kb / (kb + kc) : 0.0;
  for (int c = 0; c < 3; ++c) q[c] = m * a.rgb[c] + (1.0 - m) * q[c];
  q[3] = kb + kc;
  if (fmt == CVX_LEAF_F64) {
    double* p = (double*)pay + 4 * (uint64_t)node;
    for (int c = 0; c < 4; ++c) p[c] = q[c];
  } else {
    const double kap = fmax(q[3], 0.0);
    const uint32_t A = (uint32_t)rint(255.0 * (1.0 - exp(-kap)));
    const _Float16 h = (_Float16)(float)fmin(kap, 65504.0);
    const uint32_t hb = (uint32_t)__builtin_bit_cast(unsigned short, h);
    ((uint2*)pay)[node] =
        make_uint2(to_byte(q[0]) | (to_byte(q[1]) << 8) | (to_byte(q[2]) << 16) | (A << 24), hb);
  }
}

__global__ void k_stroke_visit(const StrokeItem* __restrict__ items, uint32_t n, StrokeArgs a,
                               const double4* __restrict__ stamps, const uint4* __restrict__ rec,
                               void* pay, uint64_t n_nodes, StrokeItem* __restrict__ next,
                               uint32_t* __restrict__ next_count, uint32_t next_cap,
                               StrokeItem* __restrict__ pend, void* __restrict__ pend_pay,
                               uint32_t* __restrict__ pend_count, uint32_t pend_cap,
                               uint32_t merge) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  StrokeItem it;
  if (items) {
    it = items[i];
  } else {  // the root array
    it.node = i;
    it.x = i % a.R;
    it.y = (i / a.R) % a.R;
    it.z = i / (a.R * a.R);
    it.depth = 0;
  }
  if (it.node >= n_nodes) return;
  const double e = ldexp(a.root_edge, -(int)it.depth);
  const double lo[3] = {a.origin[0] + (double)it.x * e, a.origin[1] + (double)it.y * e,
                        a.origin[2] + (double)it.z * e};
  bool overlap = false, inside = false;
  for (uint32_t j = 0; j < a.n_stamps; ++j) {
    const double4 s = stamps[j];
    const double rr = s.w * s.w;
    overlap = overlap || box_dist2(lo, e, s) < rr;
    inside = inside || centre_dist2(lo, e, s) <= rr;
  }
  if (!overlap) return;
  const uint32_t x = rec[it.node].x;
  if (merge) {
    // a refined cell whose 8 children are leaves with identical payloads is
    // listed (with its first child's payload); otherwise its children are
    // looked at on the next level
    if ((x & 1u) || (uint64_t)x + 8 > n_nodes) return;
    bool uni = true;
    for (uint32_t o = 0; o < 8; ++o) uni = uni && (rec[x + o].x & 1u);
    if (uni) {
      if (a.fmt == CVX_LEAF_F64) {
        const double* p0 = (const double*)pay + 4 * (uint64_t)x;
        for (uint32_t o = 1; o < 8 && uni; ++o) {
          const double* po = p0 + 4 * o;
          for (int k = 0; k < 4; ++k)
            uni = uni && __builtin_bit_cast(uint64_t, po[k]) == __builtin_bit_cast(uint64_t, p0[k]);
        }
      } else {
        const uint2 p0 = ((const uint2*)pay)[x];
        for (uint32_t o = 1; o < 8; ++o) {
          const uint2 po = ((const uint2*)pay)[x + o];
          uni = uni && po.x == p0.x && po.y == p0.y;
        }
      }
    }
    if (uni) {
      const uint32_t slot = atomicAdd(pend_count, 1u);
      if (slot < pend_cap) {
        pend[slot] = it;
        if (a.fmt == CVX_LEAF_F64) {
          const double* p0 = (const double*)pay + 4 * (uint64_t)x;
          double* q = (double*)pend_pay + 4 * (uint64_t)slot;
          for (int k = 0; k < 4; ++k) q[k] = p0[k];
        } else {
          ((uint2*)pend_pay)[slot] = ((const uint2*)pay)[x];
        }
      }
      return;
    }
  }
  if (!(x & 1u)) {
    if ((uint64_t)x + 8 > n_nodes) return;
    const uint32_t slot = atomicAdd(next_count, 8u);
    if (slot + 8 > next_cap) return;  // the host sees the count above the capacity
    for (uint32_t o = 0; o < 8; ++o) {
      StrokeItem c;
      c.node = x + o;
      c.x = 2 * it.x + (o & 1u);
      c.y = 2 * it.y + ((o >> 1) & 1u);
      c.z = 2 * it.z + ((o >> 2) & 1u);
      c.depth = it.depth + 1;
      next[slot + o] = c;
    }
    return;
  }
  if (merge) return;  // a leaf: nothing to merge below it
  if (e > a.hmin && it.depth < a.max_depth) {
    const uint32_t slot = atomicAdd(pend_count, 1u);
    if (slot < pend_cap) {
      pend[slot] = it;
      if (a.fmt == CVX_LEAF_F64) {
        const double* p = (const double*)pay + 4 * (uint64_t)it.node;
        double* q = (double*)pend_pay + 4 * (uint64_t)slot;
        for (int c = 0; c < 4; ++c) q[c] = p[c];
      } else {
        ((uint2*)pend_pay)[slot] = ((const uint2*)pay)[it.node];
      }
    }
  }
  if (inside) paint_leaf(pay, it.node, a.fmt, e, a);
}

}  // namespace

int launch_stroke_visit(void* stream, const StrokeItem* items, uint32_t n, const StrokeArgs& a,
                        const void* stamps, const void* rec, void* pay, uint64_t n_nodes,
                        StrokeItem* next, uint32_t* next_count, uint32_t next_cap,
                        StrokeItem* pend, void* pend_pay, uint32_t* pend_count, uint32_t pend_cap,
                        uint32_t merge) {
  if (!n) return hipSuccess;
  const uint32_t bs = 256;
  hipLaunchKernelGGL(k_stroke_visit, dim3((n + bs - 1) / bs), dim3(bs), 0, (hipStream_t)stream,
                     items, n, a, (const double4*)stamps, (const uint4*)rec, pay, n_nodes, next,
                     next_count, next_cap, pend, pend_pay, pend_count, pend_cap, merge);
  return (int)hipGetLastError();
}

}  // namespace cvx

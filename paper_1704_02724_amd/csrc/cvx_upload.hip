// Device re-layout of an uploaded pool and the GPU build of the 3-neighbour
// graph G_3 (Sec. 4.1.1 "Neighbor Graph", Sec. 4.1.2: G_3 is derived on the
// GPU from G_p after every update).
//
// Each cell has six face neighbours of the same or smaller depth.  The three
// on the sibling side follow from index arithmetic (the sibling across axis k
// is I xor 2^k inside the group); the three "outer" ones cross the parent's
// boundary and are stored.  They are produced level by level, one thread per
// node, from the parent's neighbours only:
//   child I = first_child(P) + o touches, on axis k, the face of P on side
//   s = bit_k(o).  Let M be P's same-depth-or-coarser neighbour across that
//   face (P's sibling when that face is inner to P's own group, P's stored
//   link otherwise, root-array arithmetic for roots).  If M is refined, the
//   same-depth neighbour of I is M's child o xor 2^k (Sec. 4.1.1: the children
//   of D_1 touching D are C(D_1) and C(D_1)+2 in the quadtree case); else M.
#include <hip/hip_runtime.h>

#include "cvx_internal.h"

namespace cvx {

__device__ __forceinline__ uint32_t neighbour_of_parent(const uint4* __restrict__ rec, uint32_t P,
                                                        uint32_t plevel, uint32_t k, uint32_t s,
                                                        uint32_t R) {
  if (plevel == 0) {
    uint32_t c[3] = {P % R, (P / R) % R, P / (R * R)};
    uint32_t stride = k == 0 ? 1u : (k == 1 ? R : R * R);
    if (s) return c[k] + 1 < R ? P + stride : CVX_NONE;
    return c[k] > 0 ? P - stride : CVX_NONE;
  }
  uint32_t oP = P & 7u;
  if (((oP >> k) & 1u) != s) return s ? P + (1u << k) : P - (1u << k);
  uint4 r = rec[P];
  return k == 0 ? r.y : (k == 1 ? r.z : r.w);
}

__global__ void k_relayout_level(const uint32_t* __restrict__ order, uint64_t begin, uint64_t end,
                                 uint32_t level, const uint2* __restrict__ raw,
                                 const void* __restrict__ raw_leaves, uint32_t fmt,
                                 uint4* __restrict__ rec, void* __restrict__ pay, uint32_t R) {
  uint64_t q = begin + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= end) return;
  uint32_t I = order[q];
  uint2 nd = raw[I];
  uint4 r;
  if (nd.x & CVX_LEAF_BIT) {
    uint32_t li = nd.x & ~CVX_LEAF_BIT;
    r.x = 1u | (level << 1);
    if (fmt == CVX_LEAF_RGBA8_F16) {
      ((uint2*)pay)[I] = ((const uint2*)raw_leaves)[li];
    } else {
      const double4* src = (const double4*)raw_leaves;
      ((double4*)pay)[I] = src[li];
    }
  } else {
    r.x = nd.x;
  }
  if (level == 0) {
    r.y = r.z = r.w = CVX_NONE;
  } else {
    uint32_t P = nd.y, o = I & 7u;
    uint32_t link[3];
    for (uint32_t k = 0; k < 3; ++k) {
      uint32_t M = neighbour_of_parent(rec, P, level - 1, k, (o >> k) & 1u, R);
      if (M != CVX_NONE) {
        uint32_t mx = rec[M].x;
        if (!(mx & 1u)) M = mx + (o ^ (1u << k));
      }
      link[k] = M;
    }
    r.y = link[0];
    r.z = link[1];
    r.w = link[2];
  }
  rec[I] = r;
}

// Top-level table (Sec. 4: the canvas is a uniform array of roots): for every
// cell of depth L, x fastest, the node of depth <= L that covers it (a leaf
// above L, or the depth-L node itself).  One thread per cell walks down from
// its root by the bits of its coordinates.
__global__ void k_top_table(const uint4* __restrict__ rec, uint64_t n_nodes, uint32_t R,
                            uint32_t L, uint32_t* __restrict__ top) {
  const uint32_t side = R << L;
  const uint64_t n = (uint64_t)side * side * side;
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t x = (uint32_t)(i % side), y = (uint32_t)((i / side) % side),
                 z = (uint32_t)(i / ((uint64_t)side * side));
  uint32_t I = (x >> L) + R * ((y >> L) + R * (z >> L));
  for (uint32_t lvl = 0; lvl < L; ++lvl) {
    const uint32_t cx = rec[I].x;
    if ((cx & 1u) || (uint64_t)cx + 8 > n_nodes) break;
    const uint32_t sh = L - 1 - lvl;
    I = cx + (((x >> sh) & 1u) | (((y >> sh) & 1u) << 1) | (((z >> sh) & 1u) << 2));
  }
  top[i] = I;
}

int launch_top_table(void* stream, const void* rec, uint64_t n_nodes, uint32_t R, uint32_t L,
                     uint32_t* top) {
  const uint64_t side = (uint64_t)R << L, n = side * side * side;
  const uint32_t bs = 256;
  hipLaunchKernelGGL(k_top_table, dim3((uint32_t)((n + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, (const uint4*)rec, n_nodes, R, L, top);
  return (int)hipGetLastError();
}

int launch_relayout_level(void* stream, const uint32_t* order, uint64_t begin, uint64_t end,
                          uint32_t level, const void* raw_nodes, const void* raw_leaves,
                          uint32_t fmt, void* rec, void* pay, uint32_t R) {
  if (end <= begin) return hipSuccess;
  const uint32_t bs = 256;
  uint64_t blocks = (end - begin + bs - 1) / bs;
  hipLaunchKernelGGL(k_relayout_level, dim3((uint32_t)blocks), dim3(bs), 0, (hipStream_t)stream,
                     order, begin, end, level, (const uint2*)raw_nodes, raw_leaves, fmt,
                     (uint4*)rec, pay, R);
  return (int)hipGetLastError();
}

}  // namespace cvx

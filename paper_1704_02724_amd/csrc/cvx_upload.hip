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

__device__ __forceinline__ uint32_t neighbour_of_parent(const uint4* rec, uint32_t P,
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

// ---- pool edits -------------------------------------------------------------
// Record words x of nodes [0, n), packed (for the host mirror).
__global__ void k_extract_x(const uint4* __restrict__ rec, uint64_t n, uint32_t* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = rec[i].x;
}

int launch_extract_x(void* stream, const void* rec, uint64_t n, uint32_t* out) {
  if (!n) return hipSuccess;
  const uint32_t bs = 256;
  hipLaunchKernelGGL(k_extract_x, dim3((uint32_t)((n + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, (const uint4*)rec, n, out);
  return (int)hipGetLastError();
}

// Record words x of touched nodes (first child, 1 | depth << 1, or CVX_FREE).
// A node that stays in the tree keeps its links (they depend on its parent,
// which did not change); a node leaving the tree gets null links.
__global__ void k_scatter_records(const uint32_t* __restrict__ ids, const uint32_t* __restrict__ xs,
                                  uint64_t n, uint4* __restrict__ rec) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t x = xs[i];
  if (x == CVX_FREE)
    rec[ids[i]] = make_uint4(CVX_FREE, CVX_NONE, CVX_NONE, CVX_NONE);
  else
    ((uint32_t*)&rec[ids[i]])[0] = x;
}

// Payloads of touched leaves, lb bytes each (8 or 32, so whole uint2 words).
__global__ void k_scatter_payloads(const uint32_t* __restrict__ ids, const uint2* __restrict__ src,
                                   uint64_t n, uint32_t words, uint2* __restrict__ pay) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * words) return;
  const uint64_t j = i / words, w = i % words;
  pay[(uint64_t)ids[j] * words + w] = src[i];
}

// One level of the G_3 rebuild: for every refined node P of the frontier
// (depth `level`, links already final), derive the outer links of its 8
// children as at upload and append the refined children to the next
// frontier.  Only the children's y, z, w words are written; the x words and
// the links of level `level` are read.
__global__ void k_links_level(const uint32_t* __restrict__ frontier, uint64_t n, uint32_t level,
                              uint4* rec, uint32_t R, uint32_t* __restrict__ next,
                              uint32_t* __restrict__ next_count, uint64_t n_nodes,
                              uint32_t* __restrict__ mark, uint32_t epoch) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t P = frontier[i];
  // a node listed twice in one frontier (reached from its parent and named
  // as a root of a changed region) is processed once
  if (mark && atomicExch(&mark[P], epoch) == epoch) return;
  const uint32_t first = rec[P].x;
  if ((first & 1u) || (uint64_t)first + 8 > n_nodes) return;
  for (uint32_t o = 0; o < 8; ++o) {
    const uint32_t C = first + o;
    uint32_t link[3];
    for (uint32_t k = 0; k < 3; ++k) {
      uint32_t M = neighbour_of_parent(rec, P, level, k, (o >> k) & 1u, R);
      if (M != CVX_NONE) {
        const uint32_t mx = rec[M].x;
        if (!(mx & 1u)) M = mx + (o ^ (1u << k));
      }
      link[k] = M;
    }
    uint32_t* w = (uint32_t*)&rec[C];
    w[1] = link[0];
    w[2] = link[1];
    w[3] = link[2];
    if (!(rec[C].x & 1u)) next[atomicAdd(next_count, 1u)] = C;
  }
}

// Roots of the regions whose links a batch of edits can change.  A node's
// links depend only on its parent's links and on the record words of the
// parent's face neighbours; so after the nodes `changed` (depth `depth`)
// were refined or coarsened, every changed link lies strictly below one of:
// a changed node that is refined (its children are new), or a refined
// same-depth face neighbour of a changed node (a sibling, a same-depth outer
// link, or at depth 0 a neighbouring root).  Outer links to coarser cells
// are leaves and have nothing below them.
__global__ void k_dirty_roots(const uint32_t* __restrict__ changed,
                              const uint32_t* __restrict__ depth, uint64_t n,
                              const uint4* __restrict__ rec, uint32_t R,
                              uint32_t* __restrict__ out, uint32_t* __restrict__ out_depth,
                              uint32_t* __restrict__ out_count, uint64_t n_nodes) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t X = changed[i], d = depth[i];
  uint32_t cand[7];
  cand[0] = X;
  if (d == 0) {
    const uint32_t c[3] = {X % R, (X / R) % R, X / (R * R)};
    for (uint32_t k = 0; k < 3; ++k) {
      const uint32_t stride = k == 0 ? 1u : (k == 1 ? R : R * R);
      cand[1 + 2 * k] = c[k] + 1 < R ? X + stride : CVX_NONE;
      cand[2 + 2 * k] = c[k] > 0 ? X - stride : CVX_NONE;
    }
  } else {
    const uint4 r = rec[X];
    for (uint32_t k = 0; k < 3; ++k) cand[1 + k] = X ^ (1u << k);
    cand[4] = r.y;
    cand[5] = r.z;
    cand[6] = r.w;
  }
  for (uint32_t j = 0; j < 7; ++j) {
    const uint32_t N = cand[j];
    if (N == CVX_NONE || (uint64_t)N >= n_nodes) continue;
    const uint32_t x = rec[N].x;
    if (x == CVX_FREE || (x & 1u)) continue;
    const uint32_t slot = atomicAdd(out_count, 1u);
    out[slot] = N;
    out_depth[slot] = d;
  }
}

int launch_dirty_roots(void* stream, const uint32_t* changed, const uint32_t* depth, uint64_t n,
                       const void* rec, uint32_t R, uint32_t* out, uint32_t* out_depth,
                       uint32_t* out_count, uint64_t n_nodes) {
  if (!n) return hipSuccess;
  const uint32_t bs = 256;
  hipLaunchKernelGGL(k_dirty_roots, dim3((uint32_t)((n + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, changed, depth, n, (const uint4*)rec, R, out, out_depth,
                     out_count, n_nodes);
  return (int)hipGetLastError();
}

int launch_scatter_records(void* stream, const uint32_t* ids, const uint32_t* xs, uint64_t n,
                           void* rec) {
  if (!n) return hipSuccess;
  const uint32_t bs = 256;
  hipLaunchKernelGGL(k_scatter_records, dim3((uint32_t)((n + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, ids, xs, n, (uint4*)rec);
  return (int)hipGetLastError();
}

int launch_scatter_payloads(void* stream, const uint32_t* ids, const void* src, uint64_t n,
                            uint32_t leaf_bytes, void* pay) {
  if (!n) return hipSuccess;
  const uint32_t bs = 256, words = leaf_bytes / 8;
  hipLaunchKernelGGL(k_scatter_payloads, dim3((uint32_t)((n * words + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, ids, (const uint2*)src, n, words, (uint2*)pay);
  return (int)hipGetLastError();
}

int launch_links_level(void* stream, const uint32_t* frontier, uint64_t n, uint32_t level,
                       void* rec, uint32_t R, uint32_t* next, uint32_t* next_count,
                       uint64_t n_nodes, uint32_t* mark, uint32_t epoch) {
  if (!n) return hipSuccess;
  const uint32_t bs = 256;
  hipLaunchKernelGGL(k_links_level, dim3((uint32_t)((n + bs - 1) / bs)), dim3(bs), 0,
                     (hipStream_t)stream, frontier, n, level, (uint4*)rec, R, next, next_count,
                     n_nodes, mark, epoch);
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

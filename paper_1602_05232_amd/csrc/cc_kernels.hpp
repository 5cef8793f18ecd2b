// Kernels of the plain (one graph, one launch set per bulk operation) path.
//
//   k_init           parent[v] = v                       (initial state, Section 4)
//   k_update_fused   Bulk-Update in one pass: both roots, then link in place
//   k_filter         Algorithm 2, relabel and filter: relabel each edge by its roots and
//                    keep the pairs whose roots differ, compacted into a live
//                    list (wavefront scan + LDS staging, one atomic per block)
//   k_link_live      join every live root pair (stands in for Algorithm 2's
//                    connected components of the contracted graph followed by
//                    Parallel-Join, Algorithm 3: CAS linking reaches the same
//                    connectivity in place and in any order)
//   k_compress_live  point the linked roots at their new root (the "pragmatic"
//                    path compression of Section 6.1, applied to the roots the
//                    minibatch touched)
//   k_query          Algorithm 1: out[i] = find(u_i) == find(v_i)
// (passes over all vertices -- labels, compression, root count -- are in
// cc_vertex_kernels.hpp)
#pragma once

#include "uf_device.hpp"

namespace ccdev {
namespace {  // kernels get internal linkage in every translation unit

__global__ void k_init(int32_t* __restrict__ parent, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t n4 = n >> 2;
  int4* p4 = reinterpret_cast<int4*>(parent);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const int32_t b = (int32_t)(i << 2);
    p4[i] = make_int4(b, b + 1, b + 2, b + 3);
  }
  for (int64_t i = (n4 << 2) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    parent[i] = (int32_t)i;
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

__device__ __forceinline__ bool in_range(int2 e, int32_t n) {
  return (uint32_t)e.x < (uint32_t)n && (uint32_t)e.y < (uint32_t)n;
}

// Block-wide exclusive scan of per-thread counts with one atomicAdd on
// *counter per block to reserve the block's output range.  Returns this
// thread's first output index.  Every thread of the block must call it.
__device__ __forceinline__ unsigned block_reserve(int cnt, unsigned* counter, int* wave_off, unsigned* blk) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int incl = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wave_off[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < nw; ++w) {
      const int c = wave_off[w];
      wave_off[w] = acc;
      acc += c;
    }
    blk[0] = acc ? atomicAdd(counter, (unsigned)acc) : 0u;
  }
  __syncthreads();
  const unsigned pos = blk[0] + (unsigned)(wave_off[wid] + incl - cnt);
  __syncthreads();  // wave_off and blk may be reused by the next call
  return pos;
}

// One tile = blockDim.x * ITEMS consecutive edges; item k of thread t is edge
// tile_start + k * blockDim.x + t, so every load instruction of a wavefront
// reads 512 contiguous bytes.  With RECORD, every root this kernel links under
// another tree is appended to `hooked` (count in hooked_ctl[0]) for the
// compression pass that follows.
template <int ITEMS, class Ord, bool RECORD>
__global__ void k_update_fused(int32_t* __restrict__ parent, const int2* __restrict__ edges, int64_t m,
                               int32_t n, unsigned long long* __restrict__ slots, int* __restrict__ flags,
                               int32_t* __restrict__ hooked, unsigned* __restrict__ hooked_ctl) {
  constexpr bool R = is_ranked<Ord>::value;
  __shared__ int wave_off[16];
  __shared__ unsigned blk[2];
  const int64_t tile = (int64_t)blockDim.x * ITEMS;
  int links = 0;
  for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < m; t0 += (int64_t)gridDim.x * tile) {
    int2 e[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t i = t0 + (int64_t)k * blockDim.x + threadIdx.x;
      e[k] = i < m ? edges[i] : make_int2(0, 0);  // padding: a self-loop on vertex 0
    }
    int32_t hk[ITEMS];
    int nh = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      hk[k] = -1;
      if (!in_range(e[k], n)) {
        raise_flag(flags, kFlagRange);
        continue;
      }
      const int32_t u = e[k].x, v = e[k].y;
      if (u == v) continue;
      const int32_t pu = ldp<R>(parent + u), pv = ldp<R>(parent + v);
      if (pu == pv || pu == v || pv == u) continue;  // already one tree
      const int32_t ru = find_halve_from<R>(parent, u, pu, n, flags);
      const int32_t rv = find_halve_from<R>(parent, v, pv, n, flags);
      if (ru != rv) {
        hk[k] = link(parent, ru, rv, n, flags, Ord{});
        if (hk[k] >= 0) ++nh;
      }
    }
    links += nh;
    if (RECORD) {
      unsigned pos = block_reserve(nh, hooked_ctl, wave_off, blk);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k)
        if (hk[k] >= 0) hooked[pos++] = hk[k];
    }
  }
  count_links(slots, links);
}

// Relabel + filter + compact.  live_ctl[0] is the live count.
template <int ITEMS>
__global__ void k_filter(int32_t* __restrict__ parent, const int2* __restrict__ edges, int64_t m, int32_t n,
                         int2* __restrict__ live, unsigned* __restrict__ live_ctl, int* __restrict__ flags) {
  extern __shared__ int2 stage[];  // blockDim.x * ITEMS pairs
  __shared__ int wave_off[16];
  __shared__ unsigned blk_base;
  __shared__ int blk_total;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int64_t tile = (int64_t)blockDim.x * ITEMS;
  for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < m; t0 += (int64_t)gridDim.x * tile) {
    int2 r[ITEMS];
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t i = t0 + (int64_t)k * blockDim.x + threadIdx.x;
      int2 e = i < m ? edges[i] : make_int2(0, 0);
      if (!in_range(e, n)) {
        raise_flag(flags, kFlagRange);
        e = make_int2(0, 0);
      }
      r[k] = e.x == e.y ? make_int2(0, 0)
                        : make_int2(find_halve(parent, e.x, n, flags), find_halve(parent, e.y, n, flags));
      cnt += r[k].x != r[k].y;
    }
    // exclusive scan of cnt over the wavefront
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    if (lane == 63) wave_off[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = 0;
      for (int w = 0; w < nw; ++w) {
        const int c = wave_off[w];
        wave_off[w] = acc;
        acc += c;
      }
      blk_total = acc;
      blk_base = acc ? atomicAdd(live_ctl, (unsigned)acc) : 0u;
    }
    __syncthreads();
    int pos = wave_off[wid] + incl - cnt;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (r[k].x != r[k].y) stage[pos++] = r[k];
    __syncthreads();
    const int total = blk_total;
    const unsigned base = blk_base;
    for (int j = threadIdx.x; j < total; j += blockDim.x) live[base + j] = stage[j];
    __syncthreads();
  }
}

template <class Ord>
__global__ void k_link_live(int32_t* __restrict__ parent, const int2* __restrict__ live,
                            const unsigned* __restrict__ live_ctl, int32_t n,
                            unsigned long long* __restrict__ slots, int* __restrict__ flags) {
  const unsigned L = __hip_atomic_load(const_cast<unsigned*>(live_ctl), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  int links = 0;
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < L; i += gridDim.x * blockDim.x) {
    const int2 p = live[i];
    links += link_roots(parent, p.x, p.y, n, flags, Ord{}) >= 0;
  }
  count_links(slots, links);
}

// Full compression of x's path: find the root, then re-walk and point each
// node at it.  Only valid while nothing is being linked.
template <bool R = false>
__device__ __forceinline__ void compress_path(int32_t* parent, int32_t x, int32_t n, int* flags) {
  const int32_t r = find_read<R>(parent, x, n, flags);
  uint32_t steps = 0;
  int32_t p = ldp<R>(parent + x);
  while (p != r && p != x) {
    st(parent + x, r);
    x = p;
    p = ldp<R>(parent + x);
    if (++steps > (uint32_t)n) break;
  }
}

// Compress the paths of both live roots.  The last block to finish clears the
// live count (live_ctl[0]) and its own completion counter (live_ctl[1]), so
// the next minibatch starts from an empty list without a host call.
__global__ void k_compress_live(int32_t* __restrict__ parent, const int2* __restrict__ live,
                                unsigned* __restrict__ live_ctl, int32_t n, int* __restrict__ flags) {
  const unsigned L = __hip_atomic_load(live_ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < L; i += gridDim.x * blockDim.x) {
    const int2 p = live[i];
    compress_path(parent, p.x, n, flags);
    compress_path(parent, p.y, n, flags);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned done =
        __hip_atomic_fetch_add(live_ctl + 1, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {
      __hip_atomic_store(live_ctl, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(live_ctl + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Compress the paths of the roots linked by the last fused update (the
// "pragmatic" compression of Section 6.1 applied to the nodes the minibatch
// changed), then the last block clears the list's count.
template <bool R = false>
__global__ void k_compress_hooked(int32_t* __restrict__ parent, const int32_t* __restrict__ hooked,
                                  unsigned* __restrict__ ctl, int32_t n, int* __restrict__ flags) {
  const unsigned L = __hip_atomic_load(ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < L; i += gridDim.x * blockDim.x)
    compress_path<R>(parent, hooked[i], n, flags);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned done = __hip_atomic_fetch_add(ctl + 1, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {
      __hip_atomic_store(ctl, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ctl + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <int ITEMS, bool HALVE, bool R = false>
__global__ void k_query(int32_t* __restrict__ parent, const int2* __restrict__ pairs, int64_t q, int32_t n,
                        uint8_t* __restrict__ out, int* __restrict__ flags) {
  const int64_t tile = (int64_t)blockDim.x * ITEMS;
  for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < q; t0 += (int64_t)gridDim.x * tile) {
    int2 e[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t i = t0 + (int64_t)k * blockDim.x + threadIdx.x;
      e[k] = i < q ? pairs[i] : make_int2(0, 0);
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t i = t0 + (int64_t)k * blockDim.x + threadIdx.x;
      uint8_t a = 0;
      if (!in_range(e[k], n)) {
        raise_flag(flags, kFlagRange);
      } else if (e[k].x == e[k].y) {
        a = 1;
      } else {
        const int32_t ru = find_root<HALVE, R>(parent, e[k].x, n, flags);
        const int32_t rv = find_root<HALVE, R>(parent, e[k].y, n, flags);
        a = ru == rv;
      }
      if (i < q) out[i] = a;
    }
  }
}

}  // namespace
}  // namespace ccdev

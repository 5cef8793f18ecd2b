// Kernels of the many-graph form: independent graphs share one parent arena
// (graph g owns ids [base_g, base_g + n_g) and its parent entries hold arena
// ids), and one launch runs one operation per graph for many graphs at once.
//
// A launch is a list of op descriptors; op i covers tiles [tile0_i,
// tile0_i + ntiles_i) of the launch's tile space, a tile being blockDim.x *
// ITEMS items.  Each block walks tiles grid-stride and looks its op up by
// binary search, so graphs of very different sizes share the grid without
// one launch per graph.  Updates and queries may be mixed in one launch:
// they touch different graphs.
#pragma once

#include "cc_kernels.hpp"
#include "cc_stream_kernels.hpp"
#include "cc_vertex_kernels.hpp"

namespace ccdev {
namespace {  // kernels get internal linkage in every translation unit

constexpr int kPoolLinkStride = 16;  // per-graph link counters 128 B apart

struct OpDesc {
  const int2* items;  // edges (update) or pairs (query), graph-local ids
  uint8_t* out;       // answers (query)
  int64_t count;
  int32_t base;       // arena offset of the graph
  int32_t n;          // vertices of the graph
  int32_t kind;       // 0 update, 1 query
  int32_t graph;      // pool slot (link counter index)
  uint32_t tile0;
  uint32_t pad;
};

__device__ __forceinline__ int find_op(const OpDesc* ops, int nops, uint32_t tile) {
  int lo = 0, hi = nops - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (ops[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int block_sum(int v, int* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  int s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;  // valid in thread 0
}

// One tile of one operation (block-uniform: every thread of the block calls it).
// HOOK: 0 id order, 1 hashed priority (of graph-local ids), 2 union by rank
// (arena ids keep each graph's local order, so ties break as in a lone graph;
// the rank bits need arena ids below 2^kRankShift).
template <int ITEMS, int HOOK, bool RECORD, bool HALVE_Q>
__device__ __forceinline__ void pool_tile(const OpDesc& op, uint32_t t, int32_t* __restrict__ arena,
                                          unsigned long long* __restrict__ glinks, int* __restrict__ flags,
                                          int32_t* __restrict__ hooked, unsigned* __restrict__ hooked_ctl,
                                          int* wave_off, unsigned* blk, int* red) {
  constexpr bool R = HOOK == 2;
  const uint32_t T = blockDim.x * ITEMS;
  const int64_t t0 = (int64_t)(t - op.tile0) * T;
  int2 e[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int64_t i = t0 + (int64_t)k * blockDim.x + threadIdx.x;
    e[k] = i < op.count ? op.items[i] : make_int2(0, 0);
  }
  if (op.kind == 0) {
    int32_t hk[ITEMS];
    int nh = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      hk[k] = -1;
      if (!in_range(e[k], op.n)) {
        raise_flag(flags, kFlagRange);
        continue;
      }
      if (e[k].x == e[k].y) continue;
      const int32_t u = op.base + e[k].x, v = op.base + e[k].y;
      const int32_t pu = ldp<R>(arena + u), pv = ldp<R>(arena + v);
      if (pu == pv || pu == v || pv == u) continue;
      const int32_t ru = find_halve_from<R>(arena, u, pu, op.n, flags);
      const int32_t rv = find_halve_from<R>(arena, v, pv, op.n, flags);
      if (ru != rv) {
        if (HOOK == 1) {
          ByHash o;
          o.base = op.base;
          hk[k] = link_roots(arena, ru, rv, op.n, flags, o);
        } else if (HOOK == 2) {
          hk[k] = link_roots_rank(arena, ru, rv, op.n, flags);
        } else {
          hk[k] = link_roots(arena, ru, rv, op.n, flags, ById{});
        }
        if (hk[k] >= 0) ++nh;
      }
    }
    const int links = block_sum(nh, red);
    if (threadIdx.x == 0 && links > 0)
      atomicAdd(glinks + (size_t)op.graph * kPoolLinkStride, (unsigned long long)links);
    if (RECORD) {
      unsigned pos = block_reserve(nh, hooked_ctl, wave_off, blk);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k)
        if (hk[k] >= 0) hooked[pos++] = hk[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t i = t0 + (int64_t)k * blockDim.x + threadIdx.x;
      uint8_t a = 0;
      if (!in_range(e[k], op.n)) {
        raise_flag(flags, kFlagRange);
      } else if (e[k].x == e[k].y) {
        a = 1;
      } else {
        const int32_t ru = find_root<HALVE_Q, R>(arena, op.base + e[k].x, op.n, flags);
        const int32_t rv = find_root<HALVE_Q, R>(arena, op.base + e[k].y, op.n, flags);
        a = ru == rv;
      }
      if (i < op.count) op.out[i] = a;
    }
  }
}

template <int ITEMS, int HOOK, bool RECORD, bool HALVE_Q>
__global__ void k_pool_phase(const OpDesc* __restrict__ ops, int nops, uint32_t ntiles,
                             int32_t* __restrict__ arena, unsigned long long* __restrict__ glinks,
                             int* __restrict__ flags, int32_t* __restrict__ hooked,
                             unsigned* __restrict__ hooked_ctl) {
  __shared__ int wave_off[16];
  __shared__ unsigned blk[2];
  __shared__ int red[16];
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const OpDesc op = ops[find_op(ops, nops, t)];
    pool_tile<ITEMS, HOOK, RECORD, HALVE_Q>(op, t, arena, glinks, flags, hooked, hooked_ctl, wave_off, blk, red);
  }
}

// Every round of a run in one cooperative launch: round r covers descriptors
// [rstart[r], rstart[r+1]) and rtiles[r] tiles; device-wide barriers keep the
// rounds in order (an operation of round r+1 may depend on one of round r on
// the same graph).  No linked-root recording in this form.
template <int ITEMS, int HOOK, bool HALVE_Q>
__global__ void k_pool_rounds(const OpDesc* __restrict__ ops, const int32_t* __restrict__ rstart,
                              const uint32_t* __restrict__ rtiles, int nrounds, int32_t* __restrict__ arena,
                              unsigned long long* __restrict__ glinks, int* __restrict__ flags, unsigned* bar,
                              unsigned spin_limit) {
  __shared__ int wave_off[16];
  __shared__ unsigned blk[2];
  __shared__ int red[16];
  unsigned gen = 0;
  for (int r = 0; r < nrounds; ++r) {
    const OpDesc* ro = ops + rstart[r];
    const int nops = rstart[r + 1] - rstart[r];
    const uint32_t ntiles = rtiles[r];
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
      const OpDesc op = ro[find_op(ro, nops, t)];
      pool_tile<ITEMS, HOOK, false, HALVE_Q>(op, t, arena, glinks, flags, nullptr, nullptr, wave_off, blk, red);
    }
    if (r + 1 < nrounds && !grid_sync(bar, gen, flags, spin_limit)) break;
  }
}

__global__ void k_init_range(int32_t* __restrict__ arena, int32_t base, int32_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    arena[base + v] = base + v;
  }
}

// Labels of one pool graph, graph-local: id order (root = minimum).
__global__ void k_pool_labels_id(int32_t* __restrict__ arena, int32_t base, int32_t n, int32_t* __restrict__ out,
                                 int* __restrict__ flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int32_t r = find_halve(arena, base + v, n, flags);
    if (ld(arena + base + v) != r) st(arena + base + v, r);
    out[v] = r - base;
  }
}

// Hashed order or rank: minimum id per root (out pre-filled with out[v] = v,
// so a root needs no atomic), then a gather.
template <bool R>
__global__ void k_pool_labels_min(int32_t* __restrict__ arena, int32_t base, int32_t n, int32_t* __restrict__ out,
                                  int* __restrict__ flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int32_t r = find_halve<R>(arena, base + v, n, flags);
    if (r == base + v) continue;
    if (ld(arena + base + v) != r) st(arena + base + v, r);
    if (ld(out + (r - base)) > v) atomicMin(out + (r - base), v);  // see k_labels_min
  }
}

template <bool R>
__global__ void k_pool_labels_gather(const int32_t* __restrict__ arena, int32_t base, int32_t n,
                                     int32_t* __restrict__ out, int* __restrict__ flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    out[v] = out[find_read<R>(arena, base + v, n, flags) - base];
  }
}

// Image conversion for save / load: arena ids <-> graph-local ids.  Done in
// unsigned arithmetic: under union by rank a root's word carries its rank in
// the top bits, and the id below them (local id + base < 2^kRankShift) never
// carries into or borrows from them.
__global__ void k_to_local(const int32_t* __restrict__ arena, int32_t base, int32_t n, int32_t* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    out[v] = (int32_t)((uint32_t)arena[base + v] - (uint32_t)base);
  }
}

// Check a graph-local image before it is placed: every entry in range and
// pointing from lower to strictly higher priority (then no cycle); count the
// roots.  res[0] = bad entries, res[1] = roots.
template <bool HASH>
__global__ void k_check_image(const int32_t* __restrict__ img, int32_t n, unsigned long long* __restrict__ res) {
  unsigned long long bad = 0, roots = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int32_t q = img[v];
    if (q < 0 || q >= n) {
      ++bad;
    } else if (q == v) {
      ++roots;
    } else if (HASH ? !(fmix32((uint32_t)q) < fmix32((uint32_t)v)) : !(q < v)) {
      ++bad;
    }
  }
  bad = (unsigned long long)wave_sum((int)bad);
  roots = (unsigned long long)wave_sum((int)roots);
  if ((threadIdx.x & 63) == 0) {
    if (bad) atomicAdd(res, bad);
    if (roots) atomicAdd(res + 1, roots);
  }
}

__global__ void k_place(const int32_t* __restrict__ img, int32_t base, int32_t n, int32_t* __restrict__ arena) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    arena[base + v] = (int32_t)((uint32_t)img[v] + (uint32_t)base);
  }
}

}  // namespace
}  // namespace ccdev

// Kernels of the many-graph form: independent graphs share one parent arena
// (graph g owns the slots [base_g, base_g + n_g), and those slots hold
// graph-local ids, so arena + base_g is graph g's own parent array), and one
// launch runs one operation per graph for many graphs at once.
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
// HOOK: 0 id order, 1 hashed priority, 2 union by rank; all on graph-local
// ids, exactly as for a lone graph (rank needs n_g below 2^kRankShift).
// With RECORD, each root this tile links is appended to `hooked` as (graph
// base, local id).
template <int ITEMS, int HOOK, bool RECORD, bool HALVE_Q>
__device__ __forceinline__ void pool_tile(const OpDesc& op, uint32_t t, int32_t* __restrict__ arena,
                                          unsigned long long* __restrict__ glinks, int* __restrict__ flags,
                                          int2* __restrict__ hooked, unsigned* __restrict__ hooked_ctl,
                                          int* wave_off, unsigned* blk, int* red) {
  constexpr bool R = HOOK == 2;
  int32_t* parent = arena + op.base;
  const uint32_t T = blockDim.x * ITEMS;
  const int64_t t0 = (int64_t)(t - op.tile0) * T;
  int2 e[ITEMS];
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const int64_t i = t0 + (int64_t)k * blockDim.x + threadIdx.x;
    e[k] = i < op.count ? ld_stream_pair(op.items, i) : make_int2(0, 0);
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
      const int32_t u = e[k].x, v = e[k].y;
      const int32_t pu = ldp<R>(parent + u), pv = ldp<R>(parent + v);
      if (pu == pv || pu == v || pv == u) continue;
      const int32_t ru = find_halve_from<R>(parent, u, pu, op.n, flags);
      const int32_t rv = find_halve_from<R>(parent, v, pv, op.n, flags);
      if (ru != rv) {
        if (HOOK == 1) hk[k] = link_roots(parent, ru, rv, op.n, flags, ByHash{});
        else if (HOOK == 2) hk[k] = link_roots_rank(parent, ru, rv, op.n, flags);
        else hk[k] = link_roots(parent, ru, rv, op.n, flags, ById{});
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
        if (hk[k] >= 0) hooked[pos++] = make_int2(op.base, hk[k]);
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
        const int32_t ru = find_root<HALVE_Q, R>(parent, e[k].x, op.n, flags);
        const int32_t rv = find_root<HALVE_Q, R>(parent, e[k].y, op.n, flags);
        a = ru == rv;
      }
      if (i < op.count) op.out[i] = a;
    }
  }
}

template <int ITEMS, int HOOK, bool RECORD, bool HALVE_Q>
__global__ void k_pool_phase(const OpDesc* __restrict__ ops, int nops, uint32_t ntiles,
                             int32_t* __restrict__ arena, unsigned long long* __restrict__ glinks,
                             int* __restrict__ flags, int2* __restrict__ hooked,
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
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    arena[base + i] = (int32_t)i;
}

// Every graph of the pool back to singletons in one pass over the arena:
// table holds (base, n) of the graphs in use, sorted by base; slot i belongs
// to the last graph whose base is at most i, if it lies within that graph.
// A block takes chunks of 16 * blockDim.x slots; one binary search per chunk
// finds the graph of its first slot, and each thread steps forward from
// there as its slots move up.  Free slots are left as they are.
__global__ void k_pool_init_all(int32_t* __restrict__ arena, int64_t capacity, const int2* __restrict__ table,
                                int count) {
  __shared__ int first;
  const int64_t chunk = (int64_t)blockDim.x * 16;
  for (int64_t c0 = (int64_t)blockIdx.x * chunk; c0 < capacity; c0 += (int64_t)gridDim.x * chunk) {
    if (threadIdx.x == 0) {
      int lo = 0, hi = count - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (table[mid].x <= c0) lo = mid; else hi = mid - 1;
      }
      first = lo;
    }
    __syncthreads();
    int g = first;
    for (int k = 0; k < 16; ++k) {
      const int64_t i = c0 + (int64_t)k * blockDim.x + threadIdx.x;
      if (i >= capacity) break;
      while (g + 1 < count && table[g + 1].x <= i) ++g;
      const int2 t = table[g];
      if (t.x <= i && i < (int64_t)t.x + t.y) arena[i] = (int32_t)(i - t.x);
    }
    __syncthreads();  // first is rewritten for the next chunk
  }
}

// Labels of one pool graph: id order (root = minimum).
__global__ void k_pool_labels_id(int32_t* __restrict__ arena, int32_t base, int32_t n, int32_t* __restrict__ out,
                                 int* __restrict__ flags) {
  int32_t* parent = arena + base;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int32_t r = find_halve(parent, v, n, flags);
    if (ld(parent + v) != r) st(parent + v, r);
    out[v] = r;
  }
}

// Hashed order or rank: minimum id per root (out pre-filled with out[v] = v,
// so a root needs no atomic), then a gather.
template <bool R>
__global__ void k_pool_labels_min(int32_t* __restrict__ arena, int32_t base, int32_t n, int32_t* __restrict__ out,
                                  int* __restrict__ flags) {
  int32_t* parent = arena + base;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int32_t r = find_halve<R>(parent, v, n, flags);
    if (r == v) continue;
    if (ld(parent + v) != r) st(parent + v, r);
    if (ld(out + r) > v) atomicMin(out + r, v);  // see k_labels_min
  }
}

template <bool R>
__global__ void k_pool_labels_gather(const int32_t* __restrict__ arena, int32_t base, int32_t n,
                                     int32_t* __restrict__ out, int* __restrict__ flags) {
  const int32_t* parent = arena + base;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    out[v] = out[find_read<R>(parent, v, n, flags)];
  }
}

// Compress the paths of the roots the last round linked, each entry (graph
// base, local id); the last block clears the list's count.
template <bool R>
__global__ void k_pool_compress_hooked(int32_t* __restrict__ arena, const int2* __restrict__ hooked,
                                       unsigned* __restrict__ ctl, int32_t cap, int* __restrict__ flags) {
  const unsigned L = __hip_atomic_load(ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < L; i += gridDim.x * blockDim.x) {
    const int2 h = hooked[i];
    compress_path<R>(arena + h.x, h.y, cap, flags);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned done = __hip_atomic_fetch_add(ctl + 1, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {
      __hip_atomic_store(ctl, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(ctl + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
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

// Check of a union-by-rank image (graph-local ids, a root's rank in the bits
// above kRankShift), which keeps no order to test edge by edge:
//   init    every entry in range, rank bits only on roots; r[v] = parent id;
//           res[0] += bad entries, res[1] += roots
//   jump    r[v] = r[r[v]] (an ancestor twice as far up, or the root); an
//           out-of-range r[v] is left alone, so a bad image cannot send a
//           read out of bounds
//   verify  after 32 jumps every vertex must have reached a root (no path is
//           2^32 long), otherwise the image holds a cycle: res[0] += 1
__global__ void k_rank_image_init(const int32_t* __restrict__ img, int32_t n, int32_t* __restrict__ r,
                                  unsigned long long* __restrict__ res) {
  unsigned long long bad = 0, roots = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i, w = img[v], q = w & kIdMask;
    if (q >= n || (w != q && q != v)) ++bad;
    roots += q == v;
    r[v] = q;
  }
  bad = (unsigned long long)wave_sum((int)bad);
  roots = (unsigned long long)wave_sum((int)roots);
  if ((threadIdx.x & 63) == 0) {
    if (bad) atomicAdd(res, bad);
    if (roots) atomicAdd(res + 1, roots);
  }
}

__global__ void k_rank_image_jump(int32_t* __restrict__ r, int32_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t q = r[i];
    if ((uint32_t)q < (uint32_t)n) r[i] = r[q];
  }
}

__global__ void k_rank_image_verify(const int32_t* __restrict__ img, const int32_t* __restrict__ r, int32_t n,
                                    unsigned long long* __restrict__ res) {
  unsigned long long bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t q = r[i];
    if ((uint32_t)q >= (uint32_t)n || (img[q] & kIdMask) != q) ++bad;
  }
  bad = (unsigned long long)wave_sum((int)bad);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(res, bad);
}

}  // namespace
}  // namespace ccdev

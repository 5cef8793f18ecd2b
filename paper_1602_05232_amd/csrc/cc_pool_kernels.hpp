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

// Membership filter of the pool (FILT).  Graph g may name an anchor vertex
// a_g (anchors[g]), and bit base_g + v of the pool's bitmap is set only once
// v is known to be connected to a_g.  Components only merge, so a set bit
// stays true for as long as the graph's forest is not reset, reloaded or
// moved; the host clears a graph's bits, anchor and anchor root before any
// of those.  Before an update round on a graph that has taken n / 8 edges or
// more since its last refresh, k_pool_filter_roots records the anchor's root
// (choosing the anchor, the first endpoint of the round's first edge, if the
// graph has none) and k_pool_filter_refresh sets the bits of that root and of
// every vertex whose parent it is, in one coalesced pass over the graph's
// slots; under union by rank most of a component hangs directly under its
// root.
// Update and query tiles only read bits: an edge or pair whose two bits are
// set is settled without a parent read.  aroot[g] < 0 means the graph has
// no bits, and its tiles skip the bitmap.

// One tile of one operation (block-uniform: every thread of the block calls it).
// HOOK: 0 id order, 1 hashed priority, 2 union by rank; all on graph-local
// ids, exactly as for a lone graph (rank needs n_g below 2^kRankShift).
// With RECORD, each root this tile links is appended to `hooked` as (graph
// base, local id).  FILT: the membership filter above.
template <int ITEMS, int HOOK, bool RECORD, bool HALVE_Q, bool FILT>
__device__ __forceinline__ void pool_tile(const OpDesc& op, uint32_t t, int32_t* __restrict__ arena,
                                          unsigned long long* __restrict__ glinks, int* __restrict__ flags,
                                          int2* __restrict__ hooked, unsigned* __restrict__ hooked_ctl,
                                          const uint32_t* __restrict__ member, const int32_t* __restrict__ aroot,
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
  // membership words of both ends, all read before any is used
  uint32_t mu[ITEMS], mv[ITEMS];
  if (FILT) {
    const bool bits = __hip_atomic_load(const_cast<int32_t*>(aroot) + op.graph, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) >= 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const bool ok = bits && in_range(e[k], op.n);
      mu[k] = ok ? bit_word(member, op.base + e[k].x) : 0u;
      mv[k] = ok ? bit_word(member, op.base + e[k].y) : 0u;
    }
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
      const bool bu = FILT && bit_test(mu[k], op.base + u), bv = FILT && bit_test(mv[k], op.base + v);
      if (bu && bv) continue;
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
      } else if (FILT && bit_test(mu[k], op.base + e[k].x) && bit_test(mv[k], op.base + e[k].y)) {
        a = 1;  // both connected to the graph's anchor
      } else {
        const int32_t ru = find_root<HALVE_Q, R>(parent, e[k].x, op.n, flags);
        const int32_t rv = find_root<HALVE_Q, R>(parent, e[k].y, op.n, flags);
        a = ru == rv;
      }
      if (i < op.count) op.out[i] = a;
    }
  }
}

template <int ITEMS, int HOOK, bool RECORD, bool HALVE_Q, bool FILT>
__global__ void k_pool_phase(const OpDesc* __restrict__ ops, int nops, uint32_t ntiles,
                             int32_t* __restrict__ arena, unsigned long long* __restrict__ glinks,
                             int* __restrict__ flags, int2* __restrict__ hooked,
                             unsigned* __restrict__ hooked_ctl, const uint32_t* __restrict__ member,
                             const int32_t* __restrict__ aroot) {
  __shared__ int wave_off[16];
  __shared__ unsigned blk[2];
  __shared__ int red[16];
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const OpDesc op = ops[find_op(ops, nops, t)];
    pool_tile<ITEMS, HOOK, RECORD, HALVE_Q, FILT>(op, t, arena, glinks, flags, hooked, hooked_ctl, member, aroot,
                                                  wave_off, blk, red);
  }
}

// Every round of a run in one cooperative launch: round r covers descriptors
// [rstart[r], rstart[r+1]) and rtiles[r] tiles; device-wide barriers keep the
// rounds in order (an operation of round r+1 may depend on one of round r on
// the same graph).  No linked-root recording in this form.  FILT: round r
// first refreshes the graphs of refresh descriptors [fstart[r],
// fstart[r+1]) of fops (ftiles[r] tiles), anchor roots and bits each
// followed by a barrier.
template <int ITEMS, int HOOK, bool HALVE_Q, bool FILT>
__global__ void k_pool_rounds(const OpDesc* __restrict__ ops, const int32_t* __restrict__ rstart,
                              const uint32_t* __restrict__ rtiles, int nrounds, int32_t* __restrict__ arena,
                              unsigned long long* __restrict__ glinks, int* __restrict__ flags, unsigned* bar,
                              unsigned spin_limit, uint32_t* __restrict__ member, int32_t* __restrict__ anchors,
                              int32_t* __restrict__ aroot, const OpDesc* __restrict__ fops,
                              const int32_t* __restrict__ fstart, const uint32_t* __restrict__ ftiles) {
  constexpr bool R = HOOK == 2;
  __shared__ int wave_off[16];
  __shared__ unsigned blk[2];
  __shared__ int red[16];
  unsigned gen = 0;
  for (int r = 0; r < nrounds; ++r) {
    if (FILT && fstart[r + 1] > fstart[r]) {  // the same in every block
      const OpDesc* fo = fops + fstart[r];
      const int nf = fstart[r + 1] - fstart[r];
      for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += gridDim.x * blockDim.x)
        filter_root_of<R>(fo[i], arena, anchors, aroot, flags);
      if (!grid_sync(bar, gen, flags, spin_limit)) break;
      for (uint32_t t = blockIdx.x; t < ftiles[r]; t += gridDim.x)
        filter_refresh_tile<R>(fo[find_op(fo, nf, t)], t, arena, member, aroot);
      if (!grid_sync(bar, gen, flags, spin_limit)) break;
    }
    const OpDesc* ro = ops + rstart[r];
    const int nops = rstart[r + 1] - rstart[r];
    const uint32_t ntiles = rtiles[r];
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
      const OpDesc op = ro[find_op(ro, nops, t)];
      pool_tile<ITEMS, HOOK, false, HALVE_Q, FILT>(op, t, arena, glinks, flags, nullptr, nullptr, member, aroot,
                                                   wave_off, blk, red);
    }
    if (r + 1 < nrounds && !grid_sync(bar, gen, flags, spin_limit)) break;
  }
}

// The filter's bits of arena slots [b0, b0 + n) cleared, and anchors[g] =
// aroot[g] = -1 for g in [g0, g1).  Device-scope stores and atomics, so that
// no other XCD's cache keeps a bit that this clears.
__global__ void k_pool_filter_clear(uint32_t* __restrict__ member, int64_t b0, int64_t n,
                                    int32_t* __restrict__ anchors, int32_t* __restrict__ aroot, int32_t g0,
                                    int32_t g1) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x, tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t g = g0 + tid; g < g1; g += stride) {
    __hip_atomic_store(anchors + g, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(aroot + g, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (n <= 0) return;
  const int64_t w0 = b0 >> 5, w1 = (b0 + n - 1) >> 5;
  for (int64_t w = w0 + tid; w <= w1; w += stride) {
    const int64_t lo = w * 32 > b0 ? w * 32 : b0, hi = w * 32 + 32 < b0 + n ? w * 32 + 32 : b0 + n;
    const int span = (int)(hi - lo), shift = (int)(lo - w * 32);
    const uint32_t mask = span == 32 ? 0xffffffffu : ((1u << span) - 1u) << shift;
    if (mask == 0xffffffffu)
      __hip_atomic_store(member + w, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      __hip_atomic_fetch_and(member + w, ~mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One graph's anchor root (one thread per refresh descriptor): choose the
// anchor if the graph has none, then record the anchor's root.
template <bool R>
__device__ __forceinline__ void filter_root_of(const OpDesc& op, const int32_t* __restrict__ arena,
                                               int32_t* __restrict__ anchors, int32_t* __restrict__ aroot,
                                               int* __restrict__ flags) {
  int32_t a = __hip_atomic_load(anchors + op.graph, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (a < 0 && op.kind == 0 && op.count > 0) {
    const int2 e = op.items[0];
    if (in_range(e, op.n) && e.x != e.y) {
      a = e.x;
      __hip_atomic_store(anchors + op.graph, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  const int32_t r = a >= 0 && a < op.n ? find_read<R>(arena + op.base, a, op.n, flags) : -1;
  __hip_atomic_store(aroot + op.graph, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One tile of a refresh (refresh descriptors count tiles of blockDim.x
// bitmap words in tile0; the graph's words are (base >> 5) ..
// ((base + n - 1) >> 5), a word possibly shared with a neighbouring graph).
// One thread per word: the word's 32 slots are one 128-byte line of the
// arena.  Sets the bits of the anchor's root and of every vertex whose
// parent it is.
template <bool R>
__device__ __forceinline__ void filter_refresh_tile(const OpDesc& op, uint32_t t, const int32_t* __restrict__ arena,
                                                    uint32_t* __restrict__ member, const int32_t* __restrict__ aroot) {
  const int32_t ra = __hip_atomic_load(const_cast<int32_t*>(aroot) + op.graph, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  if (ra < 0) return;
  const int64_t base = op.base, end = base + op.n;
  const int64_t w = (base >> 5) + (int64_t)(t - op.tile0) * blockDim.x + threadIdx.x;
  if (w > ((end - 1) >> 5)) return;
  const int64_t s0 = w * 32;
  uint32_t fresh = 0;
  if (s0 >= base && s0 + 32 <= end) {
    // two 16-byte loads in flight at a time: the one-launch form inlines this
    // beside the update tile, and eight would raise its register count (and
    // lower its cooperative grid) for a pass that is a small part of a round
    const int4* q = reinterpret_cast<const int4*>(arena + s0);
    const int32_t l0 = (int32_t)(s0 - base);
#pragma unroll 2
    for (int j = 0; j < 8; ++j) {
      const int4 x = q[j];
      const int32_t c[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (pid<R>(c[k]) == ra || l0 + 4 * j + k == ra) fresh |= 1u << (4 * j + k);
    }
  } else {
    const int64_t lo = s0 > base ? s0 : base, hi = s0 + 32 < end ? s0 + 32 : end;
    for (int64_t sl = lo; sl < hi; ++sl)
      if (pid<R>(arena[sl]) == ra || (int32_t)(sl - base) == ra) fresh |= 1u << (int)(sl - s0);
  }
  // an atomic even for a word of one graph: a plain read-modify-write could
  // write back a cached bit from before the graph was last cleared
  if (fresh) __hip_atomic_fetch_or(member + w, fresh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool R>
__global__ void k_pool_filter_roots(const OpDesc* __restrict__ ops, int nops, const int32_t* __restrict__ arena,
                                    int32_t* __restrict__ anchors, int32_t* __restrict__ aroot,
                                    int* __restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nops) filter_root_of<R>(ops[i], arena, anchors, aroot, flags);
}

template <bool R>
__global__ void k_pool_filter_refresh(const OpDesc* __restrict__ ops, int nops, uint32_t ntiles,
                                      const int32_t* __restrict__ arena, uint32_t* __restrict__ member,
                                      const int32_t* __restrict__ aroot) {
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x)
    filter_refresh_tile<R>(ops[find_op(ops, nops, t)], t, arena, member, aroot);
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

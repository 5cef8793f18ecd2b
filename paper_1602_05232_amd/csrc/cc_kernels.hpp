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
// With FILT, the fused update and the query first consult the membership
// bitmap of the largest component (cc_member_kernels.hpp).
// (passes over all vertices -- labels, compression, root count -- are in
// cc_vertex_kernels.hpp)
#pragma once

#include "cc_grid.hpp"
#include "cc_member_kernels.hpp"
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

// Joins the trees of u and v, given parent ids pu and pv read earlier (an
// earlier read may be stale; it is still an ancestor, which is all a find
// needs).  Returns the root this call linked under the other tree, or -1.
// With filt, u and v join the membership bitmap once either is known to be
// connected to the anchor (bu, bv: their bits as read before).  With a
// touched bitmap, a link marks the linked root and the vertex it now hangs
// under: every vertex that has had an edge is a non-root or a root with a
// child, and became one through such a link.
template <class Ord>
__device__ __forceinline__ int32_t settle_edge(int32_t* parent, int32_t u, int32_t v, int32_t pu, int32_t pv,
                                               int32_t n, int* flags, bool filt, int32_t ra, uint32_t* member,
                                               bool bu, bool bv, uint32_t* touched) {
  constexpr bool R = is_ranked<Ord>::value;
  if (pu == pv || pu == v || pv == u) {  // already one tree
    if (filt) member_join(member, u, v, bu, bv, bu || bv || pu == ra || pv == ra);
    return -1;
  }
  const int32_t ru = find_halve_from<R>(parent, u, pu, n, flags);
  const int32_t rv = find_halve_from<R>(parent, v, pv, n, flags);
  int32_t w = -1;
  const int32_t h = ru != rv ? link(parent, ru, rv, n, flags, Ord{}, &w) : -1;
  if (filt) member_join(member, u, v, bu, bv, bu || bv || ru == ra || rv == ra);
  if (touched && h >= 0) {
    bit_set(touched, h);
    // w now has a child.  A hub root is the winning side of many links; its
    // bit is read from L2 first so that only the first few send an atomic.
    if (!bit_test(bit_word_l2(touched, w), w)) bit_set(touched, w);
  }
  return h;
}

// Filtered form: edges the bitmap does not settle wait in a per-block LDS
// list, and the block settles the list when it is nearly full and at the
// end.  A few percent of open edges would otherwise put one slow chain of
// dependent reads (parents, finds, link) into almost every wavefront; the
// list gathers them, so the wavefronts that only stream edges and test
// bits run at the speed of those reads.  List entries carry the two bits
// read at scan time in their sign bits (ids are below 2^31).  The drain also
// keeps the touched bitmap (settle_edge).
constexpr int kDeferCap = 2048;       // entries per block (16 KB of LDS)
constexpr int kDeferTileMax = 1024;   // largest blockDim.x * ITEMS of the filtered form
constexpr int kDrainItems = 4;        // listed edges per thread per pass of the drain

template <class Ord, bool RECORD>
__device__ int drain_list(int32_t* parent, const int2* list, int nd, int32_t n, int* flags, int32_t ra,
                          uint32_t* member, uint32_t* touched, int32_t* hooked, unsigned* hooked_ctl, int* wave_off,
                          unsigned* blk) {
  constexpr bool R = is_ranked<Ord>::value;
  const int B = blockDim.x;
  int links = 0;
  for (int base = 0; base < nd; base += B * kDrainItems) {  // same trip count in every thread
    int2 p[kDrainItems];
    int32_t pu[kDrainItems], pv[kDrainItems];
    unsigned open = 0;
#pragma unroll
    for (int k = 0; k < kDrainItems; ++k) {
      const int i = base + k * B + (int)threadIdx.x;
      pu[k] = pv[k] = 0;
      p[k] = make_int2(0, 0);
      if (i < nd) {
        p[k] = list[i];
        open |= 1u << k;
        pu[k] = ldp<R>(parent + (p[k].x & 0x7fffffff));
        pv[k] = ldp<R>(parent + (p[k].y & 0x7fffffff));
      }
    }
    int32_t hk[kDrainItems];
    int nh = 0;
#pragma unroll
    for (int k = 0; k < kDrainItems; ++k) {
      hk[k] = -1;
      if (!((open >> k) & 1u)) continue;
      const int32_t u = p[k].x & 0x7fffffff, v = p[k].y & 0x7fffffff;
      hk[k] = settle_edge<Ord>(parent, u, v, pu[k], pv[k], n, flags, ra >= 0, ra, member, p[k].x < 0, p[k].y < 0,
                               touched);
      if (hk[k] >= 0) ++nh;
    }
    links += nh;
    if (RECORD) {
      unsigned pos = block_reserve(nh, hooked_ctl, wave_off, blk);
#pragma unroll
      for (int k = 0; k < kDrainItems; ++k)
        if (hk[k] >= 0) hooked[pos++] = hk[k];
    }
  }
  return links;
}

// One tile = blockDim.x * ITEMS consecutive edges; item k of thread t is edge
// tile_start + k * blockDim.x + t, so every load instruction of a wavefront
// reads 512 contiguous bytes.  With RECORD, every root this kernel links
// under another tree is appended to `hooked` (count in hooked_ctl[0]) for the
// compression pass that follows.  With FILT (blockDim.x * ITEMS at most
// kDeferTileMax), an edge whose endpoints are both in the membership bitmap
// is dropped before any parent read, the others go through the block's list
// (above), and the endpoints of every edge joined (or found joined) are added
// to the bitmap once one of them is known to be connected to the anchor.
template <int ITEMS, class Ord, bool RECORD, bool FILT>
__global__ void k_update_fused(int32_t* __restrict__ parent, const int2* __restrict__ edges, int64_t m,
                               int32_t n, unsigned long long* __restrict__ slots, int* __restrict__ flags,
                               int32_t* __restrict__ hooked, unsigned* __restrict__ hooked_ctl,
                               const int32_t* __restrict__ member_ctl, uint32_t* __restrict__ member) {
  constexpr bool R = is_ranked<Ord>::value;
  __shared__ int wave_off[17];
  __shared__ unsigned blk[2];
  __shared__ int2 list[FILT ? kDeferCap : 1];
  const int64_t tile = (int64_t)blockDim.x * ITEMS;
  const int64_t member_words = ((int64_t)n + 31) >> 5;  // the touched bitmap follows the membership bitmap
  int links = 0;
  const int32_t ra = FILT ? anchor_root<R>(parent, member_ctl, n, flags) : -1;
  const bool filt = FILT && ra >= 0;
  int nd = 0;  // FILT: entries in the block's list (the same in every thread)
  for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < m; t0 += (int64_t)gridDim.x * tile) {
    int2 e[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t i = t0 + (int64_t)k * blockDim.x + threadIdx.x;
      e[k] = i < m ? ld_stream_pair(edges, i) : make_int2(0, 0);  // padding: a self-loop on vertex 0
    }
    uint32_t mu[ITEMS], mv[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      mu[k] = mv[k] = 0u;
      if (filt && in_range(e[k], n)) {
        mu[k] = bit_word(member, e[k].x);
        mv[k] = bit_word(member, e[k].y);
      }
    }
    // With no anchor yet (a fresh forest) the bitmap can drop nothing, so
    // each edge is settled in place as in the unfiltered form, which keeps
    // the touched bitmap all the same (first R-MAT scale-24 minibatch: 0.65
    // -> 0.63 ms).
    if (FILT && filt) {
      int c = 0;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if (!in_range(e[k], n)) {
          raise_flag(flags, kFlagRange);
          e[k] = make_int2(0, 0);
          continue;
        }
        const int32_t u = e[k].x, v = e[k].y;
        const bool bu = filt && bit_test(mu[k], u), bv = filt && bit_test(mv[k], v);
        if (u == v || (bu && bv)) {
          e[k] = make_int2(0, 0);
          continue;
        }
        e[k] = make_int2(bu ? (int32_t)((uint32_t)u | 0x80000000u) : u, bv ? (int32_t)((uint32_t)v | 0x80000000u) : v);
        ++c;
      }
      int total;
      int at = nd + block_scan(c, &total, wave_off);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k)
        if (e[k].x != e[k].y) list[at++] = e[k];
      nd += total;
      if (nd > kDeferCap - (int)tile) {
        __syncthreads();  // the list is complete
        links += drain_list<Ord, RECORD>(parent, list, nd, n, flags, ra, member, member + member_words,
                                         hooked, hooked_ctl, wave_off, blk);
        __syncthreads();  // every entry has been read before the list is refilled
        nd = 0;
      }
      continue;
    }
    // Unfiltered, or filtered before an anchor exists (then the touched
    // bitmap is kept here): each item reads its parents just before it uses
    // them.
    // Reading all items' parents first measured slower under id and hashed
    // linking (8 items per thread, one large minibatch: 12.6 -> 14.0 ms and
    // 9.9 -> 13.7 ms), as the early reads go stale while earlier items link.
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
      hk[k] = settle_edge<Ord>(parent, u, v, ldp<R>(parent + u), ldp<R>(parent + v), n, flags, false, -1, member,
                               false, false, FILT ? member + member_words : nullptr);
      if (hk[k] >= 0) ++nh;
    }
    links += nh;
    if (RECORD) {
      unsigned pos = block_reserve(nh, hooked_ctl, wave_off, blk);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k)
        if (hk[k] >= 0) hooked[pos++] = hk[k];
    }
  }
  if (FILT && nd > 0) {
    __syncthreads();
    links += drain_list<Ord, RECORD>(parent, list, nd, n, flags, ra, member, member + member_words, hooked,
                                     hooked_ctl, wave_off, blk);
  }
  count_links(slots, links);
}

// Relabel + filter + compact.  live_ctl[0] is the live count.  R: root
// words carry rank bits (union by rank).
template <int ITEMS, bool R>
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
      int2 e = i < m ? ld_stream_pair(edges, i) : make_int2(0, 0);
      if (!in_range(e, n)) {
        raise_flag(flags, kFlagRange);
        e = make_int2(0, 0);
      }
      r[k] = e.x == e.y ? make_int2(0, 0)
                        : make_int2(find_halve<R>(parent, e.x, n, flags), find_halve<R>(parent, e.y, n, flags));
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
    links += link(parent, p.x, p.y, n, flags, Ord{}) >= 0;
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
template <bool R = false>
__global__ void k_compress_live(int32_t* __restrict__ parent, const int2* __restrict__ live,
                                unsigned* __restrict__ live_ctl, int32_t n, int* __restrict__ flags) {
  const unsigned L = __hip_atomic_load(live_ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < L; i += gridDim.x * blockDim.x) {
    const int2 p = live[i];
    compress_path<R>(parent, p.x, n, flags);
    compress_path<R>(parent, p.y, n, flags);
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

// Phases: touched and membership words (FILT), then the parents of the
// pairs still open, then the finds.  With FILT, while the touched bitmap is
// complete a pair with an end outside it answers 0 without a find; a pair
// whose ends are both in the membership bitmap answers 1 without a find; and
// an end whose find meets the anchor's root (or that is found joined to a
// member) is added to the membership bitmap.
template <int ITEMS, bool HALVE, bool R, bool FILT>
__global__ void k_query(int32_t* __restrict__ parent, const int2* __restrict__ pairs, int64_t q, int32_t n,
                        uint8_t* __restrict__ out, int* __restrict__ flags, const int32_t* __restrict__ member_ctl,
                        uint32_t* __restrict__ member) {
  const int64_t tile = (int64_t)blockDim.x * ITEMS;
  const int32_t ra = FILT ? anchor_root<R>(parent, member_ctl, n, flags) : -1;
  const bool filt = FILT && ra >= 0;
  const bool lone = FILT && touched_complete(member_ctl);  // the touched bitmap may prove a vertex alone
  const uint32_t* touched = FILT ? member + (((int64_t)n + 31) >> 5) : nullptr;
  for (int64_t t0 = (int64_t)blockIdx.x * tile; t0 < q; t0 += (int64_t)gridDim.x * tile) {
    int2 e[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t i = t0 + (int64_t)k * blockDim.x + threadIdx.x;
      e[k] = i < q ? ld_stream_pair(pairs, i) : make_int2(0, 0);
    }
    // While the touched bitmap is complete it holds every vertex that has
    // had an edge, members included (a member is connected to the anchor,
    // and an anchor that is still alone when picked is linked by the update
    // that follows the pick).  So the touched words go first: a clear bit
    // settles the pair as 0, and membership words are read only for pairs
    // whose ends have both had edges.  The second end's touched word is read
    // only when the first end's bit is set: fewer gathers measured faster
    // than one dependent round fewer.
    // Every lane issues each round's loads (a lane that needs no word reads
    // word 0, one line shared by the wavefront), so with several items per
    // thread the loads of a round are in flight together instead of one
    // per-item branch at a time.
    uint32_t mu[ITEMS], mv[ITEMS], tu[ITEMS], tv[ITEMS];
    bool ok[ITEMS];
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      ok[k] = in_range(e[k], n);
      mu[k] = mv[k] = 0u;
      tu[k] = tv[k] = ~0u;
    }
    if (lone) {
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) tu[k] = bit_word(touched, ok[k] ? e[k].x : 0);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const bool need = ok[k] && bit_test(tu[k], e[k].x);
        const uint32_t w = bit_word(touched, need ? e[k].y : 0);
        tv[k] = need ? w : 0u;
      }
    }
    if (filt) {
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const bool need = ok[k] && bit_test(tu[k], e[k].x) && bit_test(tv[k], e[k].y);
        const uint32_t wu = bit_word(member, need ? e[k].x : 0);
        const uint32_t wv = bit_word(member, need ? e[k].y : 0);
        mu[k] = need ? wu : 0u;
        mv[k] = need ? wv : 0u;
      }
    }
    int32_t pu[ITEMS], pv[ITEMS];
    uint8_t a[ITEMS];
    unsigned open = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      a[k] = 0;
      if (!ok[k]) {
        raise_flag(flags, kFlagRange);
        continue;
      }
      const int32_t u = e[k].x, v = e[k].y;
      if (u == v) {
        a[k] = 1;
        continue;
      }
      // an end that has never had an edge is alone, so not connected to the other
      if (!bit_test(tu[k], u) || !bit_test(tv[k], v)) continue;
      if (filt && bit_test(mu[k], u) && bit_test(mv[k], v)) {
        a[k] = 1;
        continue;
      }
      open |= 1u << k;
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {  // vertex 0 for the items already answered
      const bool o = (open >> k) & 1u;
      pu[k] = ldp<R>(parent + (o ? e[k].x : 0));
      pv[k] = ldp<R>(parent + (o ? e[k].y : 0));
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      if (!((open >> k) & 1u)) continue;
      const int32_t u = e[k].x, v = e[k].y;
      const int32_t ru = find_root_from<HALVE, R>(parent, u, pu[k], n, flags);
      const int32_t rv = find_root_from<HALVE, R>(parent, v, pv[k], n, flags);
      a[k] = ru == rv;
      if (filt) {
        const bool bu = bit_test(mu[k], u), bv = bit_test(mv[k], v);
        bool iu = bu || ru == ra, iv = bv || rv == ra;
        if (a[k]) iu = iv = iu || iv;
        if (iu && !bu) bit_set(member, u);
        if (iv && !bv) bit_set(member, v);
      }
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t i = t0 + (int64_t)k * blockDim.x + threadIdx.x;
      if (i < q) out[i] = a[k];
    }
  }
}

}  // namespace
}  // namespace ccdev

// Bulk-Find (Section 5, Algorithm 4): the roots of a whole set of vertices S,
// found together so that flows that meet are merged and every traversed node
// ends up pointing at its root (path compression shared across the set).
//
// One cooperative launch, phases separated by device-wide barriers:
//   level 0  the distinct vertices of S: a vertex is kept only on its first
//            visit (an atomic test-and-set on the visited bitmap plays
//            mkFrontier/removeDup).
//   Phase I  (read only): breadth-first search up the forest from level 0.
//            Level l + 1 holds the parents of level l's vertices that were
//            not visited before, so every visited vertex is recorded exactly
//            once; the levels together are the trail (the R_i of the
//            algorithm: a vertex's edge to its parent is parent[v] itself,
//            which Phase I does not change).
//   Phase II every trail vertex is pointed at its root.  The paper does this
//            top-down from the roots, expanding each vertex's recorded
//            children through the response distributor; on the GPU a root
//            can have millions of such children, and expanding one vertex's
//            list is serial, so Phase II here points each trail vertex at its
//            grandparent, round after round, until a round changes nothing
//            (pointer jumping restricted to the trail: O(|trail| log h)
//            work, log h rounds).  The visited bits are then cleared, so the
//            bitmap is all clear again when the kernel ends.
// The caller's operation then reads the roots with one load per vertex.
//
// Storage: level 0 goes to one segment per block (block b takes endpoints
// [b * seg0_cap, (b + 1) * seg0_cap) and keeps its first visits there).
// Levels 1, 2, ... are appended in order to one log, so that level l + 1
// occupies the log range reserved while level l was read.  A level read from
// a small predecessor (fewer than blockDim.x entries per block) is appended
// exactly, one atomic per wavefront; otherwise each block reserves chunks of
// K entries, K a power of two between blockDim.x and 1024 and at most the
// predecessor's size per block, and pads the unused tail of its last chunk
// with -1.  The padding of a level is at most one chunk per block, i.e. at
// most the size of the level before it, so the log stays below 2n entries.
//
// Bulk-Query: answer = (parent[u] == parent[v]) after the phases.
// Bulk-Update: every edge whose endpoints have different roots is linked by
// CAS (the relabel + filter of Algorithm 2 done with Bulk-Find, as Section
// 5.2 prescribes for both bulk operations).
#pragma once

#include "cc_grid.hpp"
#include "cc_kernels.hpp"

namespace ccdev {
namespace {

// ctl words: [0..1] log head (64-bit), [32], [64], [96] Phase II change flags
// (a ring of three), then the level-size groups and the barrier.
constexpr int kBfFlags = 32;
constexpr int kBfGroups = 128;
constexpr int kBfBar = kBfGroups + kCountWords;
constexpr int kBulkFindCtlWords = kBfBar + kBarWords;

struct BulkFindScratch {
  uint32_t* visited;  // n bits, all clear at rest
  int32_t* seg0;      // level 0, seg0_cap entries per block
  int32_t* log;       // levels 1, 2, ..., -1 in chunk padding
  unsigned* ctl;      // kBulkFindCtlWords, zero at launch
  int64_t seg0_cap;   // level-0 entries per block
  int64_t log_cap;    // log entries
};

// First visit of v?  A plain read skips the atomic for vertices already seen
// (hub vertices appear in many edges); the atomic decides the rest.
__device__ __forceinline__ bool test_and_set(uint32_t* bits, int32_t v) {
  const uint32_t m = 1u << (v & 31);
  if (ld((const int32_t*)bits + (v >> 5)) & (int32_t)m) return false;
  return (atomicOr(bits + (v >> 5), m) & m) == 0u;
}

// Reserve k log entries; -1 (and the corrupt flag) if the log is full, which
// the capacity bound above rules out.
__device__ __forceinline__ long long log_reserve(unsigned long long* head, int k, long long cap, int* flags) {
  const long long r = (long long)atomicAdd(head, (unsigned long long)k);
  if (r + k > cap) {
    raise_flag(flags, kFlagCorrupt);
    return -1;
  }
  return r;
}

// Append val to the log for every thread with go set.  Every thread of the
// block calls it with the same K.  K == 0: exact, one atomic per wavefront.
// Otherwise chunked: chunk[0] is the block's current chunk (-1: none) and
// chunk[1] the entries used in it; a tile's entries that do not fit go to a
// fresh chunk (a tile never exceeds one chunk, since K >= blockDim.x).
__device__ __forceinline__ void log_put(bool go, int32_t val, int32_t* log, unsigned long long* head,
                                        long long cap, int K, long long* chunk, int* wave_off, int* flags) {
  if (K == 0) {
    const unsigned long long mask = __ballot(go);
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)mask) - 1;
    long long base = 0;
    if (mask && lane == leader) base = log_reserve(head, __popcll(mask), cap, flags);
    base = __shfl(base, leader < 0 ? 0 : leader, 64);
    if (go && base >= 0) log[base + __popcll(mask & ((1ull << lane) - 1ull))] = val;
    return;
  }
  int total;
  const int off = block_scan(go ? 1 : 0, &total, wave_off);
  if (total == 0) return;
  if (threadIdx.x == 0) {
    long long b0 = chunk[0], used = chunk[1], b1 = -1;
    if (b0 < 0) {
      b0 = log_reserve(head, K, cap, flags);
      used = 0;
    }
    if (used + total > K) b1 = log_reserve(head, K, cap, flags);
    chunk[0] = b0;
    chunk[1] = used;
    chunk[2] = b1;
  }
  __syncthreads();
  const long long b0 = chunk[0], used = chunk[1], b1 = chunk[2];
  if (go) {
    const long long pos = used + off;
    const long long dst = pos < K ? (b0 < 0 ? -1 : b0 + pos) : (b1 < 0 ? -1 : b1 + pos - K);
    if (dst >= 0) log[dst] = val;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (used + total > K) {
      chunk[0] = b1;
      chunk[1] = used + total - K;
    } else {
      chunk[1] = used + total;
    }
  }
  // the next reader of chunk passes a block barrier first (the next call's
  // scan, or the barrier after the level)
}

// Point v at its grandparent; true if that changed anything.
template <bool R>
__device__ __forceinline__ bool jump(int32_t* parent, int32_t v) {
  const int32_t p = ldp<R>(parent + v);
  if (p == v) return false;
  const int32_t g = ldp<R>(parent + p);
  if (g == p) return false;
  st(parent + v, g);
  return true;
}

// items: int2 array of `count` pairs (edges or query pairs); each pair's two
// ids form S.  KIND 0 = Bulk-Update, 1 = Bulk-Query (answers to out).
template <int KIND, class Ord>
__global__ void k_bulk_find(int32_t* __restrict__ parent, const int2* __restrict__ items, int64_t count,
                            int32_t n, uint8_t* __restrict__ out, BulkFindScratch sc,
                            unsigned long long* __restrict__ slots, int* __restrict__ flags, unsigned spin_limit) {
  constexpr bool R = is_ranked<Ord>::value;
  __shared__ int wave_off[17];
  __shared__ int red;
  __shared__ long long chunk[3];
  const int B = blockDim.x, tid = threadIdx.x;
  const int64_t gsize = (int64_t)gridDim.x * B;
  const int64_t gtid = (int64_t)blockIdx.x * B + tid;
  unsigned long long* head = reinterpret_cast<unsigned long long*>(sc.ctl);
  unsigned* groups = sc.ctl + kBfGroups;
  unsigned* bar = sc.ctl + kBfBar;
  const int slot = (int)(blockIdx.x % kCountSlots) * kCountStride;
  unsigned gen = 0;

  // level 0: this block's share of the 2 * count endpoints
  const int64_t j0 = (int64_t)blockIdx.x * sc.seg0_cap;
  const int64_t j1 = j0 + sc.seg0_cap < 2 * count ? j0 + sc.seg0_cap : 2 * count;
  int32_t* seg = sc.seg0 + j0;
  int64_t cnt0 = 0;
  for (int64_t t0 = j0; t0 < j1; t0 += B) {
    const int64_t j = t0 + tid;
    int32_t v = -1;
    if (j < j1) {
      const int2 e = items[j >> 1];
      if (in_range(e, n)) v = (j & 1) ? e.y : e.x;
      else if ((j & 1) == 0) raise_flag(flags, kFlagRange);
    }
    const bool take = v >= 0 && test_and_set(sc.visited, v);
    int total;
    const int off = block_scan(take ? 1 : 0, &total, wave_off);
    if (take) seg[cnt0 + off] = v;
    cnt0 += total;
  }
  if (tid == 0 && cnt0 > 0) atomicAdd(count_group(groups, 0) + slot, (unsigned)cnt0);
  bool alive = grid_sync(bar, gen, flags, spin_limit);

  // Phase I: read level l (block-uniform loops), append level l + 1
  long long s = 0, e = 0;  // log range of level l (l >= 1)
  for (int level = 0; alive; ++level) {
    const unsigned a = group_total(count_group(groups, level), &red);
    if (a == 0u) break;
    clear_group_ahead(groups, level);
    if (level >= 1) {
      s = e;
      const long long h = (long long)__hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      e = h < sc.log_cap ? h : sc.log_cap;
    }
    int K = 0;
    const unsigned per = a / gridDim.x;
    if (per >= (unsigned)B) {
      K = B;
      while (K < 1024 && 2u * (unsigned)K <= per) K <<= 1;
    }
    if (tid == 0) {
      chunk[0] = -1;
      chunk[1] = 0;
    }
    __syncthreads();
    int outs = 0;  // this thread's appends
    const int64_t lo = level == 0 ? 0 : s, hi = level == 0 ? cnt0 : e;
    const int64_t step = level == 0 ? B : gsize, first = level == 0 ? tid : gtid;
    for (int64_t base = lo; base < hi; base += step) {
      const int64_t j = base + first;
      int32_t v = -1;
      if (j < hi) v = level == 0 ? seg[j] : sc.log[j];
      if ((uint32_t)v >= (uint32_t)n) v = -1;  // chunk padding
      int32_t p = -1;
      if (v >= 0) {
        const int32_t q = ldp<R>(parent + v);
        if (q != v && test_and_set(sc.visited, q)) p = q;
      }
      outs += p >= 0;
      log_put(p >= 0, p, sc.log, head, sc.log_cap, K, chunk, wave_off, flags);
    }
    __syncthreads();
    if (K > 0 && chunk[0] >= 0)
      for (long long t = chunk[1] + tid; t < K; t += B) sc.log[chunk[0] + t] = -1;
    const int wouts = wave_sum(outs);
    if ((tid & 63) == 0 && wouts > 0) atomicAdd(count_group(groups, level + 1) + slot, (unsigned)wouts);
    if ((int64_t)level > (int64_t)n + 1) {  // deeper than any forest
      raise_flag(flags, kFlagCorrupt);
      break;
    }
    alive = grid_sync(bar, gen, flags, spin_limit);
  }

  // Phase II: pointer jumping over the trail (own level-0 segment + the log)
  const long long hend = (long long)__hip_atomic_load(head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const long long lend = hend < sc.log_cap ? hend : sc.log_cap;
  for (int round = 0; alive; ++round) {
    if (blockIdx.x == 0 && tid == 0) st_count(sc.ctl + kBfFlags * (1 + (round + 1) % 3), 0u);
    bool moved = false;
    for (int64_t j = tid; j < cnt0; j += B) moved |= jump<R>(parent, seg[j]);
    for (int64_t j = gtid; j < lend; j += gsize) {
      const int32_t v = sc.log[j];
      if ((uint32_t)v < (uint32_t)n) moved |= jump<R>(parent, v);
    }
    if (__syncthreads_or(moved) && tid == 0) st_count(sc.ctl + kBfFlags * (1 + round % 3), 1u);
    alive = grid_sync(bar, gen, flags, spin_limit);
    if (!alive || ld_count(sc.ctl + kBfFlags * (1 + round % 3)) == 0u) break;
    if (round > 64) {  // deeper than any forest of 2^31 vertices after this many halvings
      raise_flag(flags, kFlagCorrupt);
      alive = false;
    }
  }
  for (int64_t j = tid; j < cnt0; j += B) {
    const int32_t v = seg[j];
    atomicAnd(sc.visited + (v >> 5), ~(1u << (v & 31)));
  }
  for (int64_t j = gtid; j < lend; j += gsize) {
    const int32_t v = sc.log[j];
    if ((uint32_t)v < (uint32_t)n) atomicAnd(sc.visited + (v >> 5), ~(1u << (v & 31)));
  }

  // the operation itself
  if (KIND == 1) {
    for (int64_t i = gtid; i < count; i += gsize) {
      const int2 p = items[i];
      uint8_t ans = 0;
      if (in_range(p, n)) ans = p.x == p.y || ldp<R>(parent + p.x) == ldp<R>(parent + p.y);
      out[i] = ans;
    }
  } else {
    int links = 0;
    for (int64_t i = gtid; i < count; i += gsize) {
      const int2 p = items[i];
      if (!in_range(p, n) || p.x == p.y) continue;
      const int32_t ru = ldp<R>(parent + p.x), rv = ldp<R>(parent + p.y);  // roots before any link
      if (ru != rv) links += link(parent, ru, rv, n, flags, Ord{}) >= 0;
    }
    count_links(slots, links);
  }
}

}  // namespace
}  // namespace ccdev

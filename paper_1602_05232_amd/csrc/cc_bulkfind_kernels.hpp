// Bulk-Find (Section 5, Algorithm 4): the roots of a whole set of vertices S,
// found together so that flows that meet are merged and every traversed node
// ends up pointing at its root (path compression shared across the set).
//
// One cooperative launch, phases separated by device-wide barriers:
//   Phase I  (read only): breadth-first search up the forest from S at once.
//            A vertex joins the frontier only on its first visit (an atomic
//            test-and-set on the visited bitmap plays mkFrontier/removeDup),
//            and every visited vertex is recorded once in the trail (the
//            R_i of the algorithm: its edge to the parent is parent[v] itself,
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
// Bulk-Query: answer = (parent[u] == parent[v]) after the phases.
// Bulk-Update: after one more barrier, every edge whose endpoints have
// different roots is linked by CAS (the relabel + filter of Algorithm 2 done
// with Bulk-Find, as Section 5.2 prescribes for both bulk operations).
#pragma once

#include "cc_stream_kernels.hpp"

namespace ccdev {
namespace {

struct BulkFindScratch {
  uint32_t* visited;  // n bits, all clear at rest
  int32_t* trail;     // every visited vertex once
  int32_t* f0;        // frontier ping
  int32_t* f1;        // frontier pong
  unsigned* ctl;      // [0..2] frontier counts (ring), [3] trail count,
                      // [5..7] Phase II change flags (ring),
                      // [16, 16 + kBarWords) device-wide barrier
};

// First visit of v?  A plain read skips the atomic for vertices already seen
// (hub vertices appear in many edges); the atomic decides the rest.
__device__ __forceinline__ bool test_and_set(uint32_t* bits, int32_t v) {
  const uint32_t m = 1u << (v & 31);
  if (ld((const int32_t*)bits + (v >> 5)) & (int32_t)m) return false;
  return (atomicOr(bits + (v >> 5), m) & m) == 0u;
}

constexpr int kBulkFindCtlWords = 16 + kBarWords;

// Append one item with one atomic per wavefront.
__device__ __forceinline__ unsigned wave_append(unsigned* counter, bool want) {
  const unsigned long long mask = __ballot(want);
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  unsigned base = 0;
  if (mask && lane == leader) base = atomicAdd(counter, (unsigned)__popcll(mask));
  base = __shfl(base, leader < 0 ? 0 : leader, 64);
  const unsigned below = (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
  return base + below;
}

__device__ __forceinline__ unsigned ld_count(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_count(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// items: int2 array of `count` pairs (edges or query pairs); each pair's two
// ids form S.  KIND 0 = Bulk-Update, 1 = Bulk-Query (answers to out).
template <int KIND, class Ord>
__global__ void k_bulk_find(int32_t* __restrict__ parent, const int2* __restrict__ items, int64_t count,
                            int32_t n, uint8_t* __restrict__ out, BulkFindScratch sc,
                            unsigned long long* __restrict__ slots, int* __restrict__ flags, unsigned spin_limit) {
  constexpr bool R = is_ranked<Ord>::value;
  const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned* bar = sc.ctl + 16;
  unsigned gen = 0;
  bool alive = true;

  // level 0: the distinct in-range vertices of S
  for (int64_t base = 0; base < 2 * count; base += gsize) {
    const int64_t j = base + gtid;
    int32_t v = -1;
    if (j < 2 * count) {
      const int2 e = items[j >> 1];
      if (in_range(e, n)) v = (j & 1) ? e.y : e.x;
      else if ((j & 1) == 0) raise_flag(flags, kFlagRange);
    }
    const bool take = v >= 0 && test_and_set(sc.visited, v);
    const unsigned pos = wave_append(sc.ctl + 0, take);
    if (take) sc.f0[pos] = v;
  }
  alive = grid_sync(bar, gen, flags, spin_limit);

  // Phase I
  int level = 0;
  while (alive) {
    const unsigned c = ld_count(sc.ctl + (level % 3));
    if (c == 0) break;
    if (gtid == 0) st_count(sc.ctl + ((level + 2) % 3), 0u);  // read by everyone one level ago
    const int32_t* cur = (level & 1) ? sc.f1 : sc.f0;
    int32_t* nxt = (level & 1) ? sc.f0 : sc.f1;
    unsigned* nct = sc.ctl + ((level + 1) % 3);
    for (int64_t base = 0; base < (int64_t)c; base += gsize) {
      const int64_t j = base + gtid;
      int32_t v = -1, p = -1;
      if (j < (int64_t)c) {
        v = cur[j];
        p = ldp<R>(parent + v);
      }
      const bool have = v >= 0;
      const bool is_root = have && p == v;
      const unsigned t = wave_append(sc.ctl + 3, have);
      if (have) sc.trail[t] = v;
      const bool go = have && !is_root && test_and_set(sc.visited, p);
      const unsigned q = wave_append(nct, go);
      if (go) nxt[q] = p;
    }
    ++level;
    if (level > n + 1) {
      raise_flag(flags, kFlagCorrupt);
      alive = false;
      break;
    }
    alive = grid_sync(bar, gen, flags, spin_limit);
  }

  // Phase II: pointer jumping over the trail until every trail vertex points
  // at its root.  Round r raises change flag r % 3 and clears flag (r+1) % 3,
  // which everyone read before arriving at the barrier of round r-1.
  const unsigned lam = ld_count(sc.ctl + 3);
  for (int round = 0; alive; ++round) {
    if (gtid == 0) st_count(sc.ctl + 5 + ((round + 1) % 3), 0u);
    bool moved = false;
    for (int64_t t = gtid; t < (int64_t)lam; t += gsize) {
      const int32_t v = sc.trail[t];
      const int32_t p = ldp<R>(parent + v);
      if (p == v) continue;
      const int32_t g = ldp<R>(parent + p);
      if (g != p) {
        st(parent + v, g);
        moved = true;
      }
    }
    if (moved) st_count(sc.ctl + 5 + (round % 3), 1u);
    alive = grid_sync(bar, gen, flags, spin_limit);
    if (!alive || ld_count(sc.ctl + 5 + (round % 3)) == 0u) break;
    if (round > 64) {  // deeper than any forest of 2^31 vertices after this many halvings
      raise_flag(flags, kFlagCorrupt);
      alive = false;
    }
  }
  for (int64_t t = gtid; t < (int64_t)lam; t += gsize) {
    const int32_t v = sc.trail[t];
    atomicAnd(sc.visited + (v >> 5), ~(1u << (v & 31)));
  }

  // the operation itself
  if (KIND == 1) {
    for (int64_t i = gtid; i < count; i += gsize) {
      const int2 e = items[i];
      uint8_t a = 0;
      if (in_range(e, n)) a = e.x == e.y || ldp<R>(parent + e.x) == ldp<R>(parent + e.y);
      out[i] = a;
    }
  } else {
    int links = 0;
    for (int64_t i = gtid; i < count; i += gsize) {
      const int2 e = items[i];
      if (!in_range(e, n) || e.x == e.y) continue;
      const int32_t ru = ldp<R>(parent + e.x), rv = ldp<R>(parent + e.y);  // roots before any link
      if (ru != rv) links += link(parent, ru, rv, n, flags, Ord{}) >= 0;
    }
    count_links(slots, links);
  }
}

}  // namespace
}  // namespace ccdev

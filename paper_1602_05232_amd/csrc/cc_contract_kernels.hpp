// Bulk-Update by contraction: Algorithm 2 with its connected-components step
// done on the contracted edge list itself.
//
//   relabel   (Algorithm 2, first step) every edge (u, v) becomes the pair of
//             its endpoints' roots; pairs whose roots coincide are dropped and
//             the rest are compacted into list A'' (the supernode graph).
//   round r   (the connected components of A'' and the join that follows,
//             done together in place):
//     hook      every listed pair (a, b) -- both were roots when the round
//               began -- points its lower-priority end at the other end with
//               an atomic (minimum under id order, exchange under hashed
//               order).  The atomic that still finds that end pointing at
//               itself counts one link; a later one on the same root (from
//               another pair) replaces the pointer with another
//               higher-priority vertex, which leaves a valid forest and is
//               not counted.  Nothing is retried inside the round.
//     shortcut  both ends of every pair find their current root (path
//               halving); the pair is listed for the next round only if the
//               two roots still differ.
//
// Every pointer written goes from lower to higher priority, so no cycle can
// form.  In every round the lowest-priority vertex of the list is the losing
// end of all its pairs and is hooked, so each round removes at least one root
// from the list and the rounds end (after at most as many rounds as the list
// has distinct vertices; with ids or hashes acting as random priorities the
// list shrinks geometrically in practice).  After kMaxRounds rounds whatever
// is left is joined by CAS linking (link_roots), so the launch is bounded.  Work per round is linear in the
// list, never in the original minibatch, which is what makes the form
// attractive for minibatches much larger than the number of roots they join
// (the open question of Section 7 about huge minibatches).
//
// Union by rank needs the two roots' ranks compared and the winner's rank
// raised atomically with the link, which one unconditional atomic per pair
// cannot do; the form takes the id and hashed-priority orders only.
#pragma once

#include "cc_grid.hpp"
#include "cc_kernels.hpp"

namespace ccdev {
namespace {

// The root word is read at device scope first, so that once a hook has
// landed in L2 the pairs that come later skip their atomic: a hub root is
// the losing end of very many pairs, and an L1 copy of its word would keep
// every compute unit sending it exchanges for the whole phase.
__device__ __forceinline__ int32_t ld_dev(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Hook `loser` (a root when the round began) under `winner`; 1 if this call
// was the one that took it from root to non-root.  Under id order the
// pointer only ever decreases (atomic minimum), so each root ends the round
// under the smallest of the roots it was paired with, which keeps trees
// shallow; a hashed order has no such word order and takes an exchange.
__device__ __forceinline__ int hook(int32_t* parent, int32_t loser, int32_t winner, const ById&) {
  if (ld_dev(parent + loser) <= winner) return 0;
  return atomicMin(parent + loser, winner) == loser;
}
__device__ __forceinline__ int hook(int32_t* parent, int32_t loser, int32_t winner, const ByHash&) {
  if (ld_dev(parent + loser) != loser) return 0;
  return atomicExch(parent + loser, winner) == loser;
}

// The list is split into one segment per block: block b owns edges
// [b * seg_cap, (b + 1) * seg_cap) of the minibatch and the same index range
// of `list`, keeps its survivors there (compacted in place round after
// round) and is the only block that touches them, so no list position is
// ever reserved with a global atomic.
constexpr int kContractCtlWords = kCountWords + kBarWords;
constexpr int kMaxRounds = 64;

// ctl: kContractCtlWords words, zero at launch (count groups, then barrier).
template <class Ord>
__global__ void k_contract(int32_t* __restrict__ parent, const int2* __restrict__ edges, int64_t m, int32_t n,
                           int2* __restrict__ list, int64_t seg_cap, unsigned* __restrict__ ctl,
                           unsigned long long* __restrict__ slots, int* __restrict__ flags, unsigned spin_limit) {
  constexpr int ITEMS = 4;
  __shared__ int wave_off[17];
  __shared__ int red;
  const int B = blockDim.x, tid = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * seg_cap;
  const int64_t e1 = e0 + seg_cap < m ? e0 + seg_cap : m;
  int2* seg = list + e0;
  unsigned* bar = ctl + kCountWords;
  unsigned gen = 0;
  const Ord ord{};
  const int slot = (int)(blockIdx.x % kCountSlots) * kCountStride;

  // relabel: ITEMS edges per thread per tile, each load instruction of a
  // wavefront reading 512 contiguous bytes
  int64_t cnt = 0;  // survivors of this block (uniform over the block)
  for (int64_t t0 = e0; t0 < e1; t0 += (int64_t)B * ITEMS) {
    int2 r[ITEMS];
    int c = 0;
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int64_t i = t0 + (int64_t)k * B + tid;
      r[k] = i < e1 ? ld_stream_pair(edges, i) : make_int2(0, 0);  // padding: a self-loop on vertex 0
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const int2 e = r[k];
      r[k] = make_int2(0, 0);
      if (!in_range(e, n)) {
        raise_flag(flags, kFlagRange);
      } else if (e.x != e.y) {
        const int32_t pu = ld(parent + e.x), pv = ld(parent + e.y);
        if (!(pu == pv || pu == e.y || pv == e.x))
          r[k] = make_int2(find_halve_from(parent, e.x, pu, n, flags), find_halve_from(parent, e.y, pv, n, flags));
      }
      c += r[k].x != r[k].y;
    }
    int total;
    int2* w = seg + cnt + block_scan(c, &total, wave_off);
#pragma unroll
    for (int k = 0; k < ITEMS; ++k)
      if (r[k].x != r[k].y) *w++ = r[k];
    cnt += total;
  }
  if (tid == 0 && cnt > 0) atomicAdd(count_group(ctl, 0) + slot, (unsigned)cnt);
  bool alive = grid_sync(bar, gen, flags, spin_limit);

  int links = 0;
  for (int round = 0; alive; ++round) {
    if (group_total(count_group(ctl, round), &red) == 0u) break;
    clear_group_ahead(ctl, round);

    // hook
    for (int64_t i = tid; i < cnt; i += B) {
      const int2 p = seg[i];
      const bool a_wins = ord.above(p.x, p.y);
      links += hook(parent, a_wins ? p.y : p.x, a_wins ? p.x : p.y, ord);
    }
    alive = grid_sync(bar, gen, flags, spin_limit);
    if (!alive) break;

    // shortcut + filter, compacting the segment in place: a tile's survivors
    // land at or below the tile's own positions, and the whole tile has been
    // read before the scan's first barrier lets anyone write
    int64_t kept = 0;
    for (int64_t t0 = 0; t0 < cnt; t0 += (int64_t)B * ITEMS) {
      int2 r[ITEMS];
      int c = 0;
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        const int64_t i = t0 + (int64_t)k * B + tid;
        r[k] = i < cnt ? seg[i] : make_int2(0, 0);
      }
#pragma unroll
      for (int k = 0; k < ITEMS; ++k) {
        if (r[k].x != r[k].y) r[k] = make_int2(find_halve(parent, r[k].x, n, flags), find_halve(parent, r[k].y, n, flags));
        c += r[k].x != r[k].y;
      }
      int total;
      int2* w = seg + kept + block_scan(c, &total, wave_off);
#pragma unroll
      for (int k = 0; k < ITEMS; ++k)
        if (r[k].x != r[k].y) *w++ = r[k];
      kept += total;
    }
    cnt = kept;
    if (round + 1 == kMaxRounds) {
      // Rounds always end (see above), but an adversarial order can make them
      // many; past the bound the surviving pairs are joined by CAS linking,
      // which needs no further barrier.
      for (int64_t i = tid; i < cnt; i += B) {
        const int2 p = seg[i];
        links += link_roots(parent, p.x, p.y, n, flags, ord) >= 0;
      }
      break;
    }
    if (tid == 0 && cnt > 0) atomicAdd(count_group(ctl, round + 1) + slot, (unsigned)cnt);
    alive = grid_sync(bar, gen, flags, spin_limit);
  }
  count_links(slots, links);
}

}  // namespace
}  // namespace ccdev

// Device-side union-find primitives for gfx950 (CDNA4, 64-lane wavefronts).
//
// The forest lives in one int32 parent array in HBM: parent[v] == v marks a
// root, otherwise parent[v] is v's tree parent (Section 4, union-find
// preamble).  Many threads walk and link it at once:
//
//  * Linking is a compare-and-swap of a root's own slot from "points at
//    itself" to "points at the other root" (device-scope atomic).  Only the
//    root with the LOWER priority is ever linked under the other, so every
//    parent pointer goes from lower to higher priority and no cycle can form.
//    Priority is either the vertex id (the smaller id wins, so each root is
//    the minimum id of its tree) or a hashed priority (fmix32 of the id; a
//    bijection, so there are no ties).
//  * Finds use plain loads.  Another XCD's link may not be visible yet, so a
//    find can return a vertex that WAS its root a moment ago; that is still
//    an ancestor-or-self of the true root, equal roots still prove
//    connectivity (connectivity only grows), and a link attempt on a stale
//    root fails its CAS, which returns the fresh parent to continue from.
//  * Path halving re-points each visited node at its grandparent with a
//    relaxed store.  A store only ever targets a non-root (a node seen with a
//    parent other than itself never becomes a root again) and writes one of
//    its ancestors, so it can never undo a link or create a cycle, whatever
//    order the stores land in.  The store is made at agent scope: at
//    workgroup scope such a store was measured to stay invisible to loads
//    from other XCDs well into the next kernel (Bulk-Find's first parent
//    reads returned the value from before the previous kernel's compression,
//    a few times per million trail vertices), which finds tolerate but any
//    operation that must read one parent value consistently does not.  A
//    translation unit whose forests Bulk-Find never reads (the pool's) may
//    define CC_PATH_STORE_SCOPE as workgroup scope before including this
//    header; everything here sits in an unnamed namespace, so each unit
//    keeps its own definitions.
//  * Every walk counts its steps (unsigned, so the count cannot overflow
//    before it passes n, even at n = 2^31 - 1); more than n steps means the
//    array holds a cycle, which is latched as "corrupt" and ends the walk.
//
// Kernel boundaries give each bulk operation a consistent view of the
// previous one (stream order), which realises the rule that a bulk operation
// completes before the next begins (Section 1, Model).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef CC_PATH_STORE_SCOPE
#define CC_PATH_STORE_SCOPE __HIP_MEMORY_SCOPE_AGENT
#endif

namespace ccdev {
namespace {

constexpr int kFlagRange = 1;
constexpr int kFlagCorrupt = 2;
constexpr int kFlagTimeout = 4;
constexpr int kSlots = 64;       // union counters, spread to cut atomic contention
constexpr int kSlotStride = 16;  // 16 x u64 = 128 B between counters

__device__ __forceinline__ int ld(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// A path-shortening store (halving, compression): relaxed, at the scope
// described above.
__device__ __forceinline__ void st(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, CC_PATH_STORE_SCOPE);
}
// Device-scope CAS; returns the value found (== expected on success).
__device__ __forceinline__ int32_t cas(int32_t* p, int32_t expected, int32_t desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;
}
__device__ __forceinline__ void raise_flag(int* flags, int f) {
  __hip_atomic_fetch_or(flags, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// MurmurHash3 32-bit finaliser: a bijection on 32-bit words.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// Linking orders: above(a, b) is true when a outranks b, i.e. b may be
// linked under a.  Ids may carry an offset `base` (many graphs in one array);
// the order is that of the graph-local ids, so it does not depend on where a
// graph sits.
struct ById {
  __device__ __forceinline__ bool above(int32_t a, int32_t b) const { return a < b; }
};
struct ByHash {
  int32_t base = 0;
  __device__ __forceinline__ bool above(int32_t a, int32_t b) const {
    return fmix32((uint32_t)(a - base)) < fmix32((uint32_t)(b - base));
  }
};

// Union by rank keeps each root's rank in the top bits of the root's own
// word (ids need at most kRankShift bits); a non-root word is a plain id.
// Finds under that layout mask the rank bits off (template flag R).
constexpr int kRankShift = 27;
constexpr int32_t kIdMask = (1 << kRankShift) - 1;

template <bool R>
__device__ __forceinline__ int32_t pid(int32_t w) {
  return R ? (w & kIdMask) : w;
}
template <bool R>
__device__ __forceinline__ int32_t ldp(const int32_t* p) {
  return pid<R>(ld(p));
}

// An edge or query pair, read once: a non-temporal load, so that the
// stream does not push the bitmaps and the hot parent lines out of L2
// (R-MAT scale-24 stream: update 60.5 -> 61.0 G edges/s, query 60.4 ->
// 62.8 G pairs/s).
__device__ __forceinline__ int2 ld_stream_pair(const int2* p, int64_t i) {
  const unsigned long long w = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p) + i);
  return make_int2((int32_t)(uint32_t)w, (int32_t)(uint32_t)(w >> 32));
}

// Root of x with path halving, given p = parent id of x already loaded.
template <bool R = false>
__device__ __forceinline__ int32_t find_halve_from(int32_t* parent, int32_t x, int32_t p, int32_t cap,
                                                   int* flags) {
  uint32_t steps = 0;
  while (p != x) {
    int32_t g = ldp<R>(parent + p);
    if (g == p) return p;
    st(parent + x, g);
    x = g;
    p = ldp<R>(parent + x);
    if (++steps > (uint32_t)cap) {
      raise_flag(flags, kFlagCorrupt);
      return x;
    }
  }
  return x;
}

// Root of x with path halving.
template <bool R = false>
__device__ __forceinline__ int32_t find_halve(int32_t* parent, int32_t x, int32_t cap, int* flags) {
  return find_halve_from<R>(parent, x, ldp<R>(parent + x), cap, flags);
}

// Root of x without writing, given p = parent id of x already loaded.
template <bool R = false>
__device__ __forceinline__ int32_t find_read_from(const int32_t* parent, int32_t x, int32_t p, int32_t cap,
                                                  int* flags) {
  uint32_t steps = 0;
  while (p != x) {
    x = p;
    p = ldp<R>(parent + x);
    if (++steps > (uint32_t)cap) {
      raise_flag(flags, kFlagCorrupt);
      return x;
    }
  }
  return x;
}

// Root of x without writing.
template <bool R = false>
__device__ __forceinline__ int32_t find_read(const int32_t* parent, int32_t x, int32_t cap, int* flags) {
  int32_t p = ldp<R>(parent + x);
  uint32_t steps = 0;
  while (p != x) {
    x = p;
    p = ldp<R>(parent + x);
    if (++steps > (uint32_t)cap) {
      raise_flag(flags, kFlagCorrupt);
      return x;
    }
  }
  return x;
}

template <bool HALVE, bool R = false>
__device__ __forceinline__ int32_t find_root(int32_t* parent, int32_t x, int32_t cap, int* flags) {
  if (HALVE) return find_halve<R>(parent, x, cap, flags);
  return find_read<R>(parent, x, cap, flags);
}
template <bool HALVE, bool R = false>
__device__ __forceinline__ int32_t find_root_from(int32_t* parent, int32_t x, int32_t p, int32_t cap, int* flags) {
  if (HALVE) return find_halve_from<R>(parent, x, p, cap, flags);
  return find_read_from<R>(parent, x, p, cap, flags);
}

// Join the trees whose (possibly stale) roots are a and b.  Returns the vertex
// this call linked under the other tree (a former root), or -1 if the trees
// were already one; *winner (if given) gets the root it was linked under.
template <class Ord>
__device__ __forceinline__ int32_t link_roots(int32_t* parent, int32_t a, int32_t b, int32_t cap,
                                              int* flags, const Ord& ord, int32_t* winner = nullptr) {
  uint32_t steps = 0;
  while (a != b) {
    const bool a_wins = ord.above(a, b);
    const int32_t hi = a_wins ? b : a;  // loses: gets linked under the other
    const int32_t lo = a_wins ? a : b;
    const int32_t old = cas(parent + hi, hi, lo);
    if (old == hi) {
      if (winner) *winner = lo;
      return hi;
    }
    // hi stopped being a root; continue from its current parent
    const int32_t r = find_halve(parent, old, cap, flags);
    if (a_wins) b = r; else a = r;
    if (++steps > (uint32_t)cap) {
      raise_flag(flags, kFlagCorrupt);
      return -1;
    }
  }
  return -1;
}

// Union by rank (the balanced linking of the Section 4 union-find, with
// ranks in place of sizes): the root of lower (rank, id) is linked under the
// other; on equal ranks the winner's rank then grows by one.  The CAS checks
// the loser's whole word (still a root, same rank), and a root's (rank, id)
// only grows, so keys strictly increase along every parent path: no cycle.
// A rank increment that loses a race is skipped; ranks only steer balance.
// Step bound: an unfinished pass either finds that a tracked vertex stopped
// being a root (once per vertex) or loses its CAS to a link of the loser or
// to a rank increment (each at most once per vertex: at most n - 1 links and
// n - 1 increments in a forest of n vertices), so a sound forest never needs
// 3 * cap passes, while cap passes can be too few (n = 3: CAS lost to a link,
// find, CAS lost to a link, find).
__device__ __forceinline__ int32_t link_roots_rank(int32_t* parent, int32_t a, int32_t b, int32_t cap,
                                                   int* flags, int32_t* winner = nullptr) {
  const uint64_t max_steps = 3ull * (uint64_t)(uint32_t)cap;
  uint64_t steps = 0;
  while (a != b) {
    const int32_t wa = ld(parent + a), wb = ld(parent + b);
    if ((wa & kIdMask) != a) {
      a = find_halve_from<true>(parent, a, wa & kIdMask, cap, flags);
    } else if ((wb & kIdMask) != b) {
      b = find_halve_from<true>(parent, b, wb & kIdMask, cap, flags);
    } else {
      const int32_t ra = (int32_t)((uint32_t)wa >> kRankShift), rb = (int32_t)((uint32_t)wb >> kRankShift);
      const bool a_loses = ra < rb || (ra == rb && a > b);
      const int32_t lo = a_loses ? a : b, hi = a_loses ? b : a;
      const int32_t wl = a_loses ? wa : wb, ww = a_loses ? wb : wa;
      if (cas(parent + lo, wl, hi) == wl) {
        if (ra == rb) (void)cas(parent + hi, ww, (int32_t)((uint32_t)ww + (1u << kRankShift)));
        if (winner) *winner = hi;
        return lo;
      }
    }
    if (++steps > max_steps) {
      raise_flag(flags, kFlagCorrupt);
      return -1;
    }
  }
  return -1;
}

// Marker of the rank order, and the link call for each order.
struct ByRank {};
template <class Ord>
struct is_ranked {
  static constexpr bool value = false;
};
template <>
struct is_ranked<ByRank> {
  static constexpr bool value = true;
};

template <class Ord>
__device__ __forceinline__ int32_t link(int32_t* parent, int32_t a, int32_t b, int32_t cap, int* flags,
                                        const Ord& o, int32_t* winner = nullptr) {
  return link_roots(parent, a, b, cap, flags, o, winner);
}
__device__ __forceinline__ int32_t link(int32_t* parent, int32_t a, int32_t b, int32_t cap, int* flags,
                                        const ByRank&, int32_t* winner = nullptr) {
  return link_roots_rank(parent, a, b, cap, flags, winner);
}

// Wavefront sum (64 lanes) by butterfly shuffles.
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Add this thread's successful links to one of the spread counters (one
// atomic per wavefront that linked anything).
__device__ __forceinline__ void count_links(unsigned long long* slots, int links) {
  const int tot = wave_sum(links);
  if ((threadIdx.x & 63) == 0 && tot > 0) {
    const unsigned wave = (blockIdx.x * (blockDim.x >> 6)) + (threadIdx.x >> 6);
    atomicAdd(slots + (wave % kSlots) * kSlotStride, (unsigned long long)tot);
  }
}

}  // namespace
}  // namespace ccdev

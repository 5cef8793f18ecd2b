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
//  * Path halving re-points each visited node at its grandparent with a plain
//    store.  A store only ever targets a non-root (a node seen with a parent
//    other than itself never becomes a root again) and writes one of its
//    ancestors, so it can never undo a link or create a cycle, whatever order
//    the stores land in.
//  * Every walk counts its steps; more than n steps means the array holds a
//    cycle, which is latched as "corrupt" and ends the walk.
//
// Kernel boundaries give each bulk operation a consistent view of the
// previous one (stream order), which realises the rule that a bulk operation
// completes before the next begins (Section 1, Model).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccdev {

constexpr int kFlagRange = 1;
constexpr int kFlagCorrupt = 2;
constexpr int kSlots = 64;       // union counters, spread to cut atomic contention
constexpr int kSlotStride = 16;  // 16 x u64 = 128 B between counters

__device__ __forceinline__ int ld(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void st(int32_t* p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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

// Root of x with path halving, given p = parent[x] already loaded.
__device__ __forceinline__ int32_t find_halve_from(int32_t* parent, int32_t x, int32_t p, int32_t cap,
                                                   int* flags) {
  int32_t steps = 0;
  while (p != x) {
    int32_t g = ld(parent + p);
    if (g == p) return p;
    st(parent + x, g);
    x = g;
    p = ld(parent + x);
    if (++steps > cap) {
      raise_flag(flags, kFlagCorrupt);
      return x;
    }
  }
  return x;
}

// Root of x with path halving.
__device__ __forceinline__ int32_t find_halve(int32_t* parent, int32_t x, int32_t cap, int* flags) {
  return find_halve_from(parent, x, ld(parent + x), cap, flags);
}

// Root of x without writing.
__device__ __forceinline__ int32_t find_read(const int32_t* parent, int32_t x, int32_t cap, int* flags) {
  int32_t p = ld(parent + x);
  int32_t steps = 0;
  while (p != x) {
    x = p;
    p = ld(parent + x);
    if (++steps > cap) {
      raise_flag(flags, kFlagCorrupt);
      return x;
    }
  }
  return x;
}

template <bool HALVE>
__device__ __forceinline__ int32_t find_root(int32_t* parent, int32_t x, int32_t cap, int* flags) {
  if (HALVE) return find_halve(parent, x, cap, flags);
  return find_read(parent, x, cap, flags);
}

// Join the trees whose (possibly stale) roots are a and b.  Returns the vertex
// this call linked under the other tree (a former root), or -1 if the trees
// were already one.
template <class Ord>
__device__ __forceinline__ int32_t link_roots(int32_t* parent, int32_t a, int32_t b, int32_t cap,
                                              int* flags, const Ord& ord) {
  int32_t steps = 0;
  while (a != b) {
    const bool a_wins = ord.above(a, b);
    const int32_t hi = a_wins ? b : a;  // loses: gets linked under the other
    const int32_t lo = a_wins ? a : b;
    const int32_t old = cas(parent + hi, hi, lo);
    if (old == hi) return hi;
    // hi stopped being a root; continue from its current parent
    const int32_t r = find_halve(parent, old, cap, flags);
    if (a_wins) b = r; else a = r;
    if (++steps > cap) {
      raise_flag(flags, kFlagCorrupt);
      return -1;
    }
  }
  return -1;
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

}  // namespace ccdev

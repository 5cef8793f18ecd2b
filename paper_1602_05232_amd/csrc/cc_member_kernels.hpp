// Membership filter for the largest component.
//
// A bitmap with one bit per vertex (n / 8 bytes: 2 MiB at n = 2^24, small
// enough to stay in an XCD's L2 while the parent array, 32 times larger,
// does not) records vertices known to be connected to one anchor vertex.  A
// bit is set only after a thread has seen a proof:
//
//   * the vertex's find met the anchor's root (every vertex on a parent path
//     is in the same component, so an ancestor shared with the anchor proves
//     the connection, however stale the read), or
//   * the vertex is an endpoint of an edge that this update joins (or found
//     already joined) and the other endpoint is known to be connected.
//
// Connectivity only grows (Section 4.2: the result does not depend on the
// order in which the edges of a minibatch are applied), so a set bit stays
// true for the rest of the stream.  An edge whose two endpoints both have
// their bit set can therefore be dropped without reading the parent array:
// every bit was set on the strength of edges that are linked in full by the
// end of the update, so the two ends are joined when the update completes.
// Likewise a query pair with both bits set answers 1.  This removes the two
// random parent reads for most edges late in a stream of a graph with a
// giant component (the edges that the relabel and filter of Algorithm 2
// would drop as intra-component).
//
// The anchor is chosen by k_anchor_pick, on a sparse schedule of update
// calls: it samples endpoints of the minibatch, finds their roots and takes
// the root shared by most of them.  A change of anchor to another component
// refills the membership bitmap (k_member_reseed, which first moves its bits
// into the touched bitmap below) before the update that follows.
//
// A second bitmap of the same size, `touched`, gets the bits of both ends of
// every link the filtered update makes: the root linked under another tree,
// and the vertex it then hangs under.  A vertex that has had an edge is a
// non-root or a root with a child (halving never takes a root's last child
// away), and it became one through such a link, so while every update since
// the last reset went through the filtered form (ctl[2] == 1), a vertex in
// neither bitmap has never had an edge: it is alone, and a query pairing it
// with another vertex answers 0 without a find.  Any other form of update
// clears ctl[2] (k_member_touched_invalid), and so does a load of a saved
// forest.
#pragma once

#include "uf_device.hpp"

namespace ccdev {
namespace {

constexpr int kPickThreads = 512;   // sampled edges per pick (two endpoints each)
constexpr int kPickSlots = 2048;    // LDS hash table of sampled roots
constexpr int kMemberCtlWords = 16;  // [0] anchor (-1: none), [1] refill request, [2] touched bitmap complete

// Bitmap helpers (both bitmaps): the word holding v's bit, and v's bit in
// it.  A word read before another thread set a bit only misses that bit (the
// item takes the full path), so plain loads that may hit a stale cached copy
// are fine.
__device__ __forceinline__ uint32_t bit_word(const uint32_t* bits, int32_t v) {
  return __hip_atomic_load(const_cast<uint32_t*>(bits + (v >> 5)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ bool bit_test(uint32_t word, int32_t v) { return (word >> (v & 31)) & 1u; }
// The same word read at device scope (from L2, where the atomics land).
__device__ __forceinline__ uint32_t bit_word_l2(const uint32_t* bits, int32_t v) {
  return __hip_atomic_load(const_cast<uint32_t*>(bits + (v >> 5)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void bit_set(uint32_t* bits, int32_t v) {
  __hip_atomic_fetch_or(bits + (v >> 5), 1u << (v & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The anchor's root as a kernel starts, or -1 when there is no anchor.  Later
// in the kernel it may have been linked under another root; it is then still
// an ancestor of the anchor, which is all the proofs above need.
template <bool R>
__device__ __forceinline__ int32_t anchor_root(const int32_t* parent, const int32_t* ctl, int32_t n, int* flags) {
  const int32_t a = __hip_atomic_load(const_cast<int32_t*>(ctl), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return a >= 0 && a < n ? find_read<R>(parent, a, n, flags) : -1;
}

// After u and v are known to be in one tree (joined by this thread, or found
// joined): if either is known to be connected to the anchor, so is the other.
// bu, bv: their membership bits as read earlier; in: either bit set, or
// either end's root (or parent) is the anchor's root.
__device__ __forceinline__ void member_join(uint32_t* bits, int32_t u, int32_t v, bool bu, bool bv, bool in) {
  if (!in) return;
  if (!bu) bit_set(bits, u);
  if (!bv) bit_set(bits, v);
}

__device__ __forceinline__ void pick_insert(int32_t* key, int32_t* cnt, int32_t r) {
  uint32_t h = fmix32((uint32_t)r) & (kPickSlots - 1);
  for (;;) {  // at most 2 * kPickThreads keys in kPickSlots slots: a free slot always exists
    const int32_t prev = atomicCAS(key + h, -1, r);
    if (prev == -1 || prev == r) {
      atomicAdd(cnt + h, 1);
      return;
    }
    h = (h + 1) & (kPickSlots - 1);
  }
}

// One block of kPickThreads threads.  Samples min(m, kPickThreads) evenly
// spaced edges of the minibatch about to be applied, finds the root of both
// endpoints (read-only), and counts the sampled endpoints per root.  The
// most frequent root becomes the anchor when it holds at least 1/8 of the
// sampled endpoints, at least 16 of them, and more than twice as many as the
// current anchor's component; ctl[1] then asks k_member_reseed to refill the
// bitmap, since its bits were proofs of connection to the old anchor.
template <bool R>
__global__ __launch_bounds__(kPickThreads) void k_anchor_pick(const int32_t* __restrict__ parent,
                                                              const int2* __restrict__ edges, int64_t m,
                                                              int32_t n, int32_t* __restrict__ ctl,
                                                              int* __restrict__ flags) {
  __shared__ int32_t key[kPickSlots];
  __shared__ int32_t cnt[kPickSlots];
  __shared__ unsigned long long wbest[kPickThreads / 64];
  __shared__ int whits[kPickThreads / 64];
  const int t = threadIdx.x;
  for (int i = t; i < kPickSlots; i += kPickThreads) {
    key[i] = -1;
    cnt[i] = 0;
  }
  __syncthreads();
  const int64_t s = m < kPickThreads ? m : kPickThreads;
  bool valid = false;
  if (t < s) {
    const int2 e = edges[(int64_t)t * (m / s)];
    if ((uint32_t)e.x < (uint32_t)n && (uint32_t)e.y < (uint32_t)n && e.x != e.y) {
      valid = true;
      pick_insert(key, cnt, find_read<R>(parent, e.x, n, flags));
      pick_insert(key, cnt, find_read<R>(parent, e.y, n, flags));
    }
  }
  const int total = 2 * __syncthreads_count(valid);
  const int32_t ra = anchor_root<R>(parent, ctl, n, flags);
  unsigned long long best = 0;
  int hits = 0;
  for (int i = t; i < kPickSlots; i += kPickThreads) {
    const int32_t k = key[i];
    if (k < 0) continue;
    const unsigned long long c = ((unsigned long long)(uint32_t)cnt[i] << 32) | (uint32_t)k;
    best = c > best ? c : best;
    if (k == ra) hits = cnt[i];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long o = __shfl_xor(best, off, 64);
    best = o > best ? o : best;
    hits += __shfl_xor(hits, off, 64);
  }
  if ((t & 63) == 0) {
    wbest[t >> 6] = best;
    whits[t >> 6] = hits;
  }
  __syncthreads();
  if (t == 0) {
    best = 0;
    hits = 0;
    for (int w = 0; w < kPickThreads / 64; ++w) {
      best = wbest[w] > best ? wbest[w] : best;
      hits += whits[w];
    }
    const int bc = (int)(best >> 32);
    const int32_t bk = (int32_t)(uint32_t)best;
    const bool change = total > 0 && bk != ra && bc >= 16 && 8 * bc >= total && bc > 2 * hits;
    if (change) ctl[0] = bk;
    ctl[1] = change ? 1 : 0;
  }
}

// When the last pick changed the anchor (ctl[1] != 0): moves every
// membership bit into the touched bitmap (a member has had an edge, or is
// about to get one in the update that follows its pick; a touched bit that
// is set without need only costs a find) and refills the membership bitmap
// with what one coalesced pass over `parent` proves: the new anchor's root
// and every vertex whose parent it is.  Under union by rank most of a
// component hangs directly under its root, so the update that follows starts
// with most of the component known instead of an empty bitmap.  A wavefront
// covers 64 consecutive vertices, two bitmap words, which its ballot fills.
// bits: `words` membership words followed by `words` touched words.
template <bool R>
__global__ void k_member_reseed(const int32_t* __restrict__ parent, int32_t n, const int32_t* __restrict__ ctl,
                                uint32_t* __restrict__ bits, int64_t words, int* __restrict__ flags) {
  if (__hip_atomic_load(const_cast<int32_t*>(ctl + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
  const int32_t ra = anchor_root<R>(parent, ctl, n, flags);
  uint32_t* touched = bits + words;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  constexpr int G = 4;  // 64-vertex groups per wavefront per pass, their loads in flight together
  // blockDim.x is a multiple of 64 and every wavefront starts at a multiple of
  // 64, so `i - lane` (the group's first vertex) is the same in all its lanes
  for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 - lane < n; i0 += G * stride) {
    int32_t p[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int64_t i = i0 + k * stride;
      p[k] = i < n ? pid<R>(parent[i]) : -1;
    }
    // the two word-writing lanes of each group: its new words, then all the
    // old words read together, then the writes
    uint32_t fresh[G];
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int64_t i = i0 + k * stride;
      const bool in = i < n && ra >= 0 && (i == ra || p[k] == ra);
      const unsigned long long mask = __ballot(in);  // groups past n give 0 and are not written
      fresh[k] = lane == 0 ? (uint32_t)mask : (uint32_t)(mask >> 32);
    }
    if (lane == 0 || lane == 32) {
      uint32_t old[G];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int64_t w = (i0 + k * stride) >> 5;  // the word of this lane's 32 vertices
        old[k] = w < words ? __hip_atomic_load(bits + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
      }
      // device-scope stores: this clears bits, and a cleared bit that
      // another XCD still read as set would be a false proof
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int64_t w = (i0 + k * stride) >> 5;
        if (w >= words) continue;
        if (old[k]) __hip_atomic_fetch_or(touched + w, old[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(bits + w, fresh[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// No anchor, no request, and whether the (separately cleared) touched bitmap
// describes the forest: 1 for the initial forest, 0 after a load.
__global__ void k_member_ctl_reset(int32_t* __restrict__ ctl, int touched_complete) {
  if (threadIdx.x < kMemberCtlWords) ctl[threadIdx.x] = threadIdx.x == 0 ? -1 : threadIdx.x == 2 ? touched_complete : 0;
}

// An update that does not maintain the touched bitmap is about to run.
__global__ void k_member_touched_invalid(int32_t* __restrict__ ctl) {
  if (threadIdx.x == 0) ctl[2] = 0;
}

// Ask the next k_member_reseed to refill the membership bitmap although the
// anchor stayed (Bulk-Find sets no bits of its own).
__global__ void k_member_request_refill(int32_t* __restrict__ ctl) {
  if (threadIdx.x == 0) __hip_atomic_store(ctl + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool touched_complete(const int32_t* ctl) {
  return __hip_atomic_load(const_cast<int32_t*>(ctl + 2), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

}  // namespace
}  // namespace ccdev

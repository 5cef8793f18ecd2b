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
//   Phase II every trail vertex is pointed at its root, in one of two ways
//            (template PH2):
//            0  pointer jumping restricted to the trail: every trail vertex
//               is pointed at its grandparent, round after round, until a
//               round changes nothing (O(|trail| log h) work, log h rounds);
//            1  the paper's top-down distribution through the response
//               distributor (Section 5.1): the pairs (parent(x), x) of the
//               trail's non-roots are sorted by a hash of parent(x) into
//               3 * lambda buckets (counting sort: histogram, scan, scatter)
//               with an offset array; then, level by level from the roots,
//               every vertex v that has its root r hands r to allFrom(v), the
//               pairs in v's bucket whose first entry is v (O(|trail|)
//               expected work).  A bucket of up to kRdThread pairs is read by
//               one thread, a longer one by a block, a hub's bucket (more
//               than kRdGrid pairs) by the whole grid, so that a root with
//               millions of recorded children does not serialise one thread.
//            The visited bits are then cleared, so the bitmap is all clear
//            again when the kernel ends.
// The caller's operation then reads the roots with one load per vertex.
//
// With the membership filter (member != null), an item whose two ends are
// both known to be connected to the filter's anchor is settled without a
// find: its ends never enter level 0, a query pair of that kind answers 1
// and an edge of that kind links nothing.  The membership bits are read,
// never written, in this kernel; the caller renews them (cc_plain.hip).
// The touched bitmap (member + words, every vertex that has had an edge) is
// kept by Bulk-Update: both ends of every edge it does not settle are
// marked (a settled edge's ends are members, which have had edges).  While
// the device flag says it is complete (ctl[2]), a Bulk-Query pair with an
// end that never had an edge is settled as well: it answers whether its two
// ids are equal.
//
// Storage: level 0 runs as a kernel of its own (k_bulk_find_level0, an
// ordinary launch as wide as the items want, with no device-wide barrier),
// one segment per block of that launch: block b takes items
// [b * seg0_cap / 2, (b + 1) * seg0_cap / 2), keeps the first visits of
// their ends in [b * seg0_cap, (b + 1) * seg0_cap) and writes how many in
// seg_n[2 b] (a Bulk-Update's open items: seg_n[2 b + 1]).  The cooperative
// kernel that follows (k_bulk_find) reads segments b, b + G, b + 2G, ... in
// its block b, G its own grid, which can then be narrower: every barrier
// of Phases I and II costs more the more blocks it has.
// Levels 1, 2, ... are appended in order to one log, so that level l + 1
// occupies the log range reserved while level l was read.  Each level
// reserves through a counter of its own (a ring of three, cleared two
// levels ahead), counted from the end of the level before it: once a level
// is complete its end is fixed, although the fastest blocks are already
// reserving the next level's entries while the slowest are still reading
// where the complete one ends.  A level read from a small predecessor (fewer
// than blockDim.x entries per block) is appended exactly, one atomic per
// wavefront; otherwise each block reserves chunks of K entries, K a power of
// two between blockDim.x and 1024 and at most the predecessor's size per
// block, and pads the unused tail of its last chunk with -1.  The padding of
// a level is at most one chunk per block, i.e. at most the size of the level
// before it, so the log stays below 2n entries.  The top-down list of the
// response distributor is kept the same way.
//
// The response distributor reads each trail vertex's parent several times
// (Phase I, the bucket count, the scatter) and needs the same value every
// time, or a pair lands outside the bucket range its count reserved.  That
// holds: parent words change within the launch only in the top-down phase,
// and earlier launches store them at agent scope (see uf_device.hpp).
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

// ctl words (all zero at launch, every counter on a 128-byte line of its
// own): [0], [32], [64] the log's per-level reservation counters (64-bit, a
// ring of three), [96], [128], [160] Phase II change flags (a ring of three),
// then the level-size groups and the barrier, then the response
// distributor's words: [0], [32], [64] the top-down list's per-level
// reservation counters (64-bit, a ring of three), [96], [128], [160] heads of
// the per-level list of buckets one block serves (a ring of three), [192],
// [224], [256] entries appended per level without padding (a ring of three),
// [288], [320], [352] heads of the per-level list of buckets the whole grid
// serves (a ring of three), [384 ..] one partial sum per block (the bucket
// scan; at most kRdMaxBlocks blocks).
constexpr int kBfLevels = 0;
constexpr int kBfFlags = 96;
constexpr int kBfGroups = 192;
constexpr int kBfBar = kBfGroups + kCountWords;
constexpr int kBfRd = kBfBar + kBarWords;
constexpr int kRdMaxBlocks = 1024;
constexpr int kBulkFindCtlWords = kBfRd + 384 + kRdMaxBlocks;
static_assert(kBfRd % 2 == 0, "64-bit counters need 8-byte alignment");

// Counter of ring r (0, 1, 2) at ctl + at, 32 words apart.
__device__ __forceinline__ unsigned* ring_word(unsigned* ctl, int at, int r) { return ctl + at + 32 * (r % 3); }
__device__ __forceinline__ unsigned long long* ring_ctr(unsigned* ctl, int at, int r) {
  return reinterpret_cast<unsigned long long*>(ring_word(ctl, at, r));
}
__device__ __forceinline__ unsigned long long ld_ctr(unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void clear_ctr(unsigned long long* p) {
  __hip_atomic_store(p, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Where one level's entries go: base + the level's own counter, below cap.
struct LevelOut {
  unsigned long long* ctr;
  long long base;
  long long cap;
};

// Root entries of the top-down list are appended in chunks of kRdRootChunk
// per block (one atomic per chunk: exact appends, one atomic per wavefront
// on the one counter, took 0.4 ms of a 1.4 ms query call on the R-MAT
// stream).  A block's last chunk is padded, so the list holds up to
// kRdRootPad more entries: blocks of 256 threads, at most 1024 of them.
constexpr int kRdRootChunk = 512;
constexpr int64_t kRdRootPad = 1024 * (int64_t)kRdRootChunk;

// Bucket sizes served by one thread, and above which the whole grid serves
// a bucket (between the two: one block).
constexpr int kRdThread = 16;
constexpr int64_t kRdGrid = 1 << 15;

struct BulkFindScratch {
  uint32_t* visited;  // n bits, all clear at rest
  int32_t* seg0;      // level 0, seg0_cap entries per level-0 block
  uint32_t* open;     // Bulk-Update: seg0_cap / 2 entries per level-0 block, the items left open (or null)
  uint32_t* seg_n;    // 2 per level-0 block: entries of its segment, then its open items
  int64_t seg_blocks; // blocks of the level-0 launch
  int32_t* log;       // levels 1, 2, ..., -1 in chunk padding
  unsigned* ctl;      // kBulkFindCtlWords, zero at launch
  int64_t seg0_cap;   // level-0 entries per block
  int64_t log_cap;    // log entries
  // response distributor (PH2 = 1), rd_cap >= level-0 entries + log entries
  uint32_t* rd_cnt;   // 3 * rd_cap + 1: bucket counts, then scatter cursors
  uint32_t* rd_off;   // 3 * rd_cap + 1: bucket offsets
  int2* rd_pairs;     // rd_cap: (parent(x), x), sorted by bucket
  int2* rd_down;      // 2 * rd_cap + kRdRootPad: (vertex, root) of the top-down levels, (-1, -1) in chunk padding
  int32_t* rd_big;    // rd_cap: top-down entries whose bucket a block serves (from the front) or the grid
                      // serves (from the back); together at most one level's entries
  int64_t rd_cap;
};

// Bucket of `from` among rho buckets (a 64-bit mix, then a multiply-high).
__device__ __forceinline__ uint64_t rd_bucket(int32_t from, uint64_t rho) {
  uint64_t h = (uint64_t)(uint32_t)from * 0x9e3779b97f4a7c15ull;
  h ^= h >> 29;
  h *= 0xbf58476d1ce4e5b9ull;
  h ^= h >> 32;
  return __umul64hi(h, rho);
}

// First visit of v?  A read skips the atomic for vertices already seen (hub
// vertices appear in many edges); the atomic decides the rest.  Within a
// call bits are only set until the clearing at its end, so a read that
// misses another block's fresh bit only costs the atomic.
__device__ __forceinline__ bool test_and_set(uint32_t* bits, int32_t v) {
  const uint32_t m = 1u << (v & 31);
  if (bits[v >> 5] & m) return false;
  return (atomicOr(bits + (v >> 5), m) & m) == 0u;
}

// Reserve k entries of a level; -1 (and the corrupt flag) if the list is
// full, which the capacity bounds rule out.
__device__ __forceinline__ long long level_reserve(const LevelOut& lv, int k, int* flags) {
  const long long r = lv.base + (long long)atomicAdd(lv.ctr, (unsigned long long)k);
  if (r + k > lv.cap) {
    raise_flag(flags, kFlagCorrupt);
    return -1;
  }
  return r;
}

// Append val to the level's list for every thread with go set.  Every
// thread of the block calls it with the same K.  K == 0: exact, one atomic
// per wavefront.  Otherwise chunked: chunk[0] is the block's current chunk
// (-1: none) and chunk[1] the entries used in it; a tile's entries that do
// not fit go to a fresh chunk (a tile never exceeds one chunk, since
// K >= blockDim.x).  The caller pads the unused tail of the last chunk.
template <class T>
__device__ __forceinline__ void level_put(bool go, T val, T* list, const LevelOut& lv, int K, long long* chunk,
                                          int* wave_off, int* flags) {
  if (K == 0) {
    const unsigned long long mask = __ballot(go);
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)mask) - 1;
    long long base = 0;
    if (mask && lane == leader) base = level_reserve(lv, __popcll(mask), flags);
    base = __shfl(base, leader < 0 ? 0 : leader, 64);
    if (go && base >= 0) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = val;
    return;
  }
  int total;
  const int off = block_scan(go ? 1 : 0, &total, wave_off);
  if (total == 0) return;
  if (threadIdx.x == 0) {
    long long b0 = chunk[0], used = chunk[1], b1 = -1;
    if (b0 < 0) {
      b0 = level_reserve(lv, K, flags);
      used = 0;
    }
    if (used + total > K) b1 = level_reserve(lv, K, flags);
    chunk[0] = b0;
    chunk[1] = used;
    chunk[2] = b1;
  }
  __syncthreads();
  const long long b0 = chunk[0], used = chunk[1], b1 = chunk[2];
  if (go) {
    const long long pos = used + off;
    const long long dst = pos < K ? (b0 < 0 ? -1 : b0 + pos) : (b1 < 0 ? -1 : b1 + pos - K);
    if (dst >= 0) list[dst] = val;
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

// Add 1 to cnt[k] for every lane with go set and return the value before the
// add (the lane's slot).  Every lane of the wavefront calls it.  Lanes that
// share a key are served by one atomic: twice the key of the first pending
// lane is matched across the wavefront (a hub's bucket, that millions of trail
// vertices point into, is then one atomic per wavefront instead of one per
// vertex: served one at a time at one address, those dominated the call);
// lanes left after that add one by one.
__device__ __forceinline__ uint32_t bucket_add(uint32_t* cnt, uint64_t k, bool go) {
  const int lane = threadIdx.x & 63;
  const unsigned long long below = (1ull << lane) - 1ull;
  uint32_t slot = 0;
  bool pending = go;
#pragma unroll
  for (int round = 0; round < 2; ++round) {
    const unsigned long long mask = __ballot(pending);
    if (mask == 0ull) break;
    const int leader = __ffsll((long long)mask) - 1;
    const uint64_t kl = __shfl(k, leader, 64);
    const unsigned long long same = __ballot(pending && k == kl);
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt + kl, (uint32_t)__popcll(same));
    base = __shfl(base, leader, 64);
    if (pending && k == kl) {
      slot = base + (uint32_t)__popcll(same & below);
      pending = false;
    }
  }
  if (pending) slot = atomicAdd(cnt + k, 1u);
  return slot;
}

// Histogram of one pair (p, .) per lane with go set: the block's hot parent
// is counted in shared memory (hot_ctr[0], one add per wavefront), any
// other through bucket_add.  Every lane of the wavefront calls it.
__device__ __forceinline__ void hist_add(uint32_t* cnt, int32_t p, uint64_t rho, bool go, int32_t hot,
                                         unsigned* hot_ctr) {
  const bool h = go && p == hot;
  const unsigned long long hm = __ballot(h);
  if (hm && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)hm) - 1)) atomicAdd(hot_ctr, (unsigned)__popcll(hm));
  (void)bucket_add(cnt, go && !h ? rd_bucket(p, rho) : 0, go && !h);
}

// Scatter slot of one pair per lane with go set: the block's hot parent's
// pairs fill the block's reserved range (base hot_ctr[2], cursor
// hot_ctr[1]), any other takes its bucket's cursor through bucket_add.
// Every lane of the wavefront calls it.
__device__ __forceinline__ uint32_t scatter_slot(uint32_t* cnt, int32_t p, uint64_t rho, bool go, int32_t hot,
                                                 unsigned* hot_ctr) {
  const int lane = threadIdx.x & 63;
  const bool h = go && p == hot;
  const unsigned long long hm = __ballot(h);
  uint32_t hb = 0;
  if (hm) {
    const int leader = __ffsll((long long)hm) - 1;
    if (lane == leader) hb = atomicAdd(hot_ctr + 1, (unsigned)__popcll(hm));
    hb = __shfl(hb, leader, 64);
  }
  const uint32_t at = bucket_add(cnt, go && !h ? rd_bucket(p, rho) : 0, go && !h);
  return h ? hot_ctr[2] + hb + (uint32_t)__popcll(hm & ((1ull << lane) - 1ull)) : at;
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

// Both ends of an in-range item known to be connected to the anchor.
__device__ __forceinline__ bool both_members(const uint32_t* member, int2 p) {
  return member && bit_test(bit_word(member, p.x), p.x) && bit_test(bit_word(member, p.y), p.y);
}

// A query pair with an end that never had an edge (touched complete).
__device__ __forceinline__ bool lone_end(const uint32_t* touched, int2 p) {
  return touched && !(bit_test(bit_word(touched, p.x), p.x) && bit_test(bit_word(touched, p.y), p.y));
}

// Mark v as having had an edge (read first: most are marked already).
__device__ __forceinline__ void mark_touched(uint32_t* touched, int32_t v) {
  if (!bit_test(bit_word_l2(touched, v), v)) bit_set(touched, v);
}

// Both kernels below take items, an int2 array of `count` pairs (edges or
// query pairs) whose ids form S (less the items the membership bits
// settle), and KIND 0 = Bulk-Update, 1 = Bulk-Query (answers to out).
constexpr uint8_t kBfOpen = 2;  // a query pair left open by level 0, answered after Phase II
constexpr int kBfLevel0MaxBlocks = 4096;  // blocks of a level-0 launch at most
constexpr int kBfCoopBlocks = 256;        // blocks of the cooperative launch at most

// Level 0: every item read once, one thread per item.  An item settled here
// (out of range, a self-loop, proved by the bitmaps) gets a query answer
// now, an open one the mark kBfOpen, and its ends' first visits go to the
// block's segment.  touched_bits: the touched bitmap, read by queries while
// the device says it is complete.
template <int KIND>
__global__ void k_bulk_find_level0(const int2* __restrict__ items, int64_t count, int32_t n,
                                   uint8_t* __restrict__ out, BulkFindScratch sc, int* __restrict__ flags,
                                   const uint32_t* __restrict__ member, const uint32_t* __restrict__ touched_bits,
                                   const int32_t* __restrict__ member_ctl) {
  __shared__ int wave_off[17];
  const int B = blockDim.x, tid = threadIdx.x;
  const uint32_t* touched = KIND == 1 && touched_bits && touched_complete(member_ctl) ? touched_bits : nullptr;
  const int64_t per = sc.seg0_cap >> 1;
  const int64_t i0 = (int64_t)blockIdx.x * per;
  const int64_t i1 = i0 + per < count ? i0 + per : count;
  int32_t* seg = sc.seg0 + 2 * i0;
  int64_t cnt0 = 0;
  // Bulk-Update: the block's open items, listed for the linking at the end
  uint32_t* open = KIND == 0 ? sc.open : nullptr;
  int64_t nopen = 0;
  for (int64_t t0 = i0; t0 < i1; t0 += B) {
    const int64_t i = t0 + tid;
    int32_t a = -1, b = -1;
    if (i < i1) {
      const int2 e = items[i];
      if (!in_range(e, n)) {
        raise_flag(flags, kFlagRange);
        if (KIND == 1) out[i] = 0;
      } else if (e.x == e.y) {
        if (KIND == 1) out[i] = 1;  // an edge from a vertex to itself changes nothing
      } else if (KIND == 1 && lone_end(touched, e)) {
        out[i] = 0;
      } else if (both_members(member, e)) {
        if (KIND == 1) out[i] = 1;
      } else {
        if (KIND == 1) out[i] = kBfOpen;
        a = e.x;
        b = e.y;
      }
    }
    const bool ta = a >= 0 && test_and_set(sc.visited, a);
    const bool tb = b >= 0 && test_and_set(sc.visited, b);
    // one scan for both counts: kept ends in the low 16 bits (at most 2 per
    // thread and 2048 per pass), open items above
    const bool op = open && a >= 0;
    int total;
    const int off = block_scan((int)ta + (int)tb + ((int)op << 16), &total, wave_off);
    if (ta) seg[cnt0 + (off & 0xffff)] = a;
    if (tb) seg[cnt0 + (off & 0xffff) + (ta ? 1 : 0)] = b;
    if (op) open[i0 + nopen + (off >> 16)] = (uint32_t)i;
    cnt0 += total & 0xffff;
    nopen += total >> 16;
  }
  if (tid == 0) {
    sc.seg_n[2 * blockIdx.x] = (uint32_t)cnt0;
    sc.seg_n[2 * blockIdx.x + 1] = (uint32_t)nopen;
    const int slot = (int)(blockIdx.x % kCountSlots) * kCountStride;
    if (cnt0 > 0) atomicAdd(count_group(sc.ctl + kBfGroups, 0) + slot, (unsigned)cnt0);
  }
}

// Calls f(v) for every entry v of the level-0 segments this block reads
// (segments blockIdx.x, + gridDim.x, ...), in block-uniform loops: every
// thread calls f the same number of times, with v = -1 past a segment's end.
template <class F>
__device__ __forceinline__ void for_level0(const BulkFindScratch& sc, F&& f) {
  const int64_t per = sc.seg0_cap >> 1;
  for (int64_t a = blockIdx.x; a < sc.seg_blocks; a += gridDim.x) {
    const int32_t* seg = sc.seg0 + 2 * a * per;
    const int64_t cnt = sc.seg_n[2 * a];
    for (int64_t base = 0; base < cnt; base += blockDim.x) {
      const int64_t j = base + threadIdx.x;
      f(j < cnt ? seg[j] : -1);
    }
  }
}

// Phases I and II and the operation itself, one cooperative launch after
// k_bulk_find_level0 (whose writes the launch boundary publishes).
template <int KIND, class Ord, int PH2>
__global__ void k_bulk_find(int32_t* __restrict__ parent, const int2* __restrict__ items, int64_t count,
                            int32_t n, uint8_t* __restrict__ out, BulkFindScratch sc,
                            unsigned long long* __restrict__ slots, int* __restrict__ flags, unsigned spin_limit,
                            const uint32_t* __restrict__ member, uint32_t* __restrict__ touched_bits) {
  constexpr bool R = is_ranked<Ord>::value;
  __shared__ int wave_off[17];
  __shared__ int red;
  __shared__ long long chunk[3];
  __shared__ int32_t hot_key[17];   // response distributor: per-wavefront candidates, [16] the block's hot parent
  __shared__ int hot_votes[16];
  __shared__ unsigned hot_ctr[3];   // hot pairs counted, placed, and the base of the block's range
  __shared__ int pass_max[16];      // top-down phase A: longest short bucket per wavefront
  const int B = blockDim.x, tid = threadIdx.x;
  const int64_t gsize = (int64_t)gridDim.x * B;
  const int64_t gtid = (int64_t)blockIdx.x * B + tid;
  unsigned* groups = sc.ctl + kBfGroups;
  unsigned* bar = sc.ctl + kBfBar;
  const int slot = (int)(blockIdx.x % kCountSlots) * kCountStride;
  unsigned gen = 0;
  bool alive = true;

  // Phase I: read level l (block-uniform loops), append level l + 1 at the
  // end of level l's log range
  long long s = 0, e = 0;  // log range of level l (l >= 1); level 1 starts at 0
  unsigned total0 = 0;     // level-0 entries of all blocks
  for (int level = 0; alive; ++level) {
    const unsigned a = group_total(count_group(groups, level), &red);
    if (level == 0) total0 = a;
    if (a == 0u) break;
    clear_group_ahead(groups, level);
    if (level >= 1) {
      s = e;
      const long long h = s + (long long)ld_ctr(ring_ctr(sc.ctl, kBfLevels, level));
      e = h < sc.log_cap ? h : sc.log_cap;
    }
    // the counter level + 2 reserves through was last read at the start of
    // level - 1, which every block has passed
    if (blockIdx.x == 0 && tid == 0) clear_ctr(ring_ctr(sc.ctl, kBfLevels, level + 2));
    const LevelOut next{ring_ctr(sc.ctl, kBfLevels, level + 1), e, sc.log_cap};
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
    // one step up from v (-1: none), called by every thread alike
    auto climb = [&](int32_t v) {
      if ((uint32_t)v >= (uint32_t)n) v = -1;  // chunk padding
      int32_t p = -1;
      if (v >= 0) {
        const int32_t q = ldp<R>(parent + v);
        if (q != v && test_and_set(sc.visited, q)) p = q;
      }
      outs += p >= 0;
      level_put(p >= 0, p, sc.log, next, K, chunk, wave_off, flags);
    };
    if (level == 0) {
      for_level0(sc, climb);
    } else {
      for (int64_t base = s; base < e; base += gsize) {
        const int64_t j = base + gtid;
        climb(j < e ? sc.log[j] : -1);
      }
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
  // the log ends with the last non-empty level (an empty level reserved
  // nothing)
  const long long lend = e;

  if (PH2 == 1) {
    // Phase II through the response distributor.  lam bounds the pairs (the
    // trail, log padding included); rho = 3 * lam buckets.
    const long long lam = (long long)total0 + lend;
    const uint64_t rho = 3ull * (uint64_t)(lam > 0 ? lam : 1);
    uint32_t* cnt = sc.rd_cnt;
    uint32_t* off = sc.rd_off;
    unsigned* blk = sc.ctl + kBfRd + 384;
    const long long dcap = 2 * sc.rd_cap + kRdRootPad;
    if (tid == 0) {
      chunk[0] = -1;
      chunk[1] = 0;
    }
    // (a) clear the bucket counts.  Each block also picks its hot parent:
    //     the parent that most of its first entries point at (a hub root
    //     with millions of trail children).  The block counts and places
    //     the pairs under it through shared memory, with one device atomic
    //     per phase, where even per-wavefront combining left tens of
    //     thousands of atomics on that one bucket (histogram and scatter
    //     0.4 ms each of a 1.7 ms query call on the R-MAT stream).  Any
    //     choice is correct: the histogram and the scatter read the same
    //     items and the same parents, so they agree on which are hot.
    for (int64_t i = gtid; i <= (int64_t)rho; i += gsize) cnt[i] = 0u;
    {
      const int64_t per0 = sc.seg0_cap >> 1;
      const int64_t cnt_first = blockIdx.x < sc.seg_blocks ? (int64_t)sc.seg_n[2 * blockIdx.x] : 0;
      const int32_t v = tid < cnt_first ? sc.seg0[2 * blockIdx.x * per0 + tid] : -1;
      const int32_t p = v >= 0 ? ldp<R>(parent + v) : -1;
      const bool go = v >= 0 && p != v;
      const unsigned long long m = __ballot(go);
      int32_t key = -1;
      int votes = 0;
      if (m) {
        const int leader = __ffsll((long long)m) - 1;
        key = __shfl(p, leader, 64);
        votes = __popcll(__ballot(go && p == key));
      }
      if ((tid & 63) == 0) {
        hot_key[tid >> 6] = key;
        hot_votes[tid >> 6] = votes;
      }
      __syncthreads();
      if (tid == 0) {
        int best = 0;
        for (int w = 1; w < (B >> 6); ++w)
          if (hot_votes[w] > hot_votes[best]) best = w;
        hot_key[16] = hot_votes[best] >= 8 ? hot_key[best] : -1;
        hot_ctr[0] = 0u;  // hot pairs counted (histogram)
        hot_ctr[1] = 0u;  // hot pairs placed (scatter)
      }
      __syncthreads();
    }
    const int32_t hot = hot_key[16];
    alive = alive && grid_sync(bar, gen, flags, spin_limit);
    // (b) histogram of the pairs by bucket; the roots form level 0 of the
    //     top-down list (chunks of kRdRootChunk per block, the real count
    //     in the level's ring word)
    const LevelOut roots{ring_ctr(sc.ctl, kBfRd, 0), 0, dcap};
    int nroots = 0;
    if (alive)
      for_level0(sc, [&](int32_t v) {
        const int32_t p = v >= 0 ? ldp<R>(parent + v) : -1;
        hist_add(cnt, p, rho, v >= 0 && p != v, hot, hot_ctr);
        nroots += v >= 0 && p == v;
        level_put(v >= 0 && p == v, make_int2(v, v), sc.rd_down, roots, kRdRootChunk, chunk, wave_off, flags);
      });
    for (int64_t base = 0; alive && base < lend; base += gsize) {
      const int64_t j = base + gtid;
      int32_t v = j < lend ? sc.log[j] : -1;
      if ((uint32_t)v >= (uint32_t)n) v = -1;
      const int32_t p = v >= 0 ? ldp<R>(parent + v) : -1;
      hist_add(cnt, p, rho, v >= 0 && p != v, hot, hot_ctr);
      nroots += v >= 0 && p == v;
      level_put(v >= 0 && p == v, make_int2(v, v), sc.rd_down, roots, kRdRootChunk, chunk, wave_off, flags);
    }
    __syncthreads();
    if (chunk[0] >= 0)
      for (long long t = chunk[1] + tid; t < kRdRootChunk; t += B) sc.rd_down[chunk[0] + t] = make_int2(-1, -1);
    {
      int block_roots;
      (void)block_scan(nroots, &block_roots, wave_off);
      if (tid == 0 && block_roots > 0) atomicAdd(ring_word(sc.ctl, kBfRd + 192, 0), (unsigned)block_roots);
    }
    if (tid == 0 && hot >= 0 && hot_ctr[0] > 0u) atomicAdd(cnt + rd_bucket(hot, rho), hot_ctr[0]);
    alive = alive && grid_sync(bar, gen, flags, spin_limit);
    // (c) exclusive scan of the counts into the offsets: block b scans its
    //     chunk of buckets after the partial sums of the blocks before it
    const int64_t nb = (int64_t)rho + 1;
    const int64_t per = (nb + gridDim.x - 1) / gridDim.x;
    const int64_t c0 = (int64_t)blockIdx.x * per < nb ? (int64_t)blockIdx.x * per : nb;
    const int64_t c1 = c0 + per < nb ? c0 + per : nb;
    if (alive) {
      int part = 0;
      for (int64_t i = c0 + tid; i < c1; i += B) part += (int)cnt[i];
      int tot;
      (void)block_scan(part, &tot, wave_off);
      if (tid == 0) st_count(blk + blockIdx.x, (unsigned)tot);
    }
    alive = alive && grid_sync(bar, gen, flags, spin_limit);
    if (alive) {
      int pre = 0;
      for (int b = tid; b < (int)blockIdx.x; b += B) pre += (int)ld_count(blk + b);
      int tot;
      (void)block_scan(pre, &tot, wave_off);
      unsigned run = (unsigned)tot;  // sum of the blocks before this one
      for (int64_t t0 = c0; t0 < c1; t0 += B) {
        const int64_t i = t0 + tid;
        const int c = i < c1 ? (int)cnt[i] : 0;
        int tile;
        const int o = block_scan(c, &tile, wave_off);
        if (i < c1) {
          off[i] = run + (unsigned)o;
          cnt[i] = run + (unsigned)o;  // scatter cursor
        }
        run += (unsigned)tile;
      }
    }
    alive = alive && grid_sync(bar, gen, flags, spin_limit);
    // (d) scatter the pairs into their buckets (block- and grid-uniform
    //     trip counts: the slot helpers are collective over the wavefront);
    //     the block's hot pairs fill a range it reserves with one atomic
    if (tid == 0) hot_ctr[2] = (alive && hot >= 0 && hot_ctr[0] > 0u) ? atomicAdd(cnt + rd_bucket(hot, rho), hot_ctr[0]) : 0u;
    __syncthreads();
    if (alive)
      for_level0(sc, [&](int32_t v) {
        const int32_t p = v >= 0 ? ldp<R>(parent + v) : -1;
        const bool go = v >= 0 && p != v;
        const uint32_t at = scatter_slot(cnt, p, rho, go, hot, hot_ctr);
        if (go) sc.rd_pairs[at] = make_int2(p, v);
      });
    for (int64_t base = 0; alive && base < lend; base += gsize) {
      const int64_t j = base + gtid;
      int32_t v = j < lend ? sc.log[j] : -1;
      if ((uint32_t)v >= (uint32_t)n) v = -1;
      const int32_t p = v >= 0 ? ldp<R>(parent + v) : -1;
      const bool go = v >= 0 && p != v;
      const uint32_t at = scatter_slot(cnt, p, rho, go, hot, hot_ctr);
      if (go) sc.rd_pairs[at] = make_int2(p, v);
    }
    alive = alive && grid_sync(bar, gen, flags, spin_limit);
    // (e) top-down: level i = list range [ds, de); every (v, r) hands r to
    //     the pairs (v, u) of v's bucket, which point u at r and form level
    //     i + 1, appended from de on.  Short buckets are read by the entry's
    //     thread, longer ones by a block or (hubs) by the grid.
    long long ds = 0, de = 0;
    if (alive) {
      const long long h = (long long)ld_ctr(roots.ctr);
      de = h < dcap ? h : dcap;
    }
    long long real = alive ? (long long)ld_count(ring_word(sc.ctl, kBfRd + 192, 0)) : 0;  // level 0's entries without padding
    for (int level = 0; alive && de > ds; ++level) {
      unsigned* bighead = ring_word(sc.ctl, kBfRd + 96, level);
      unsigned* hubhead = ring_word(sc.ctl, kBfRd + 288, level);
      unsigned* realnext = ring_word(sc.ctl, kBfRd + 192, level + 1);
      const LevelOut next{ring_ctr(sc.ctl, kBfRd, level + 1), de, dcap};
      // chunks of K per block, K at most the current level's entries per
      // block, so a level's padding (one partial chunk per block) is at most
      // the level before it without its padding: the list stays below twice
      // the trail
      int K = 0;
      const long long perb = real / gridDim.x;
      int mine = 0;  // this thread's appends in this level
      if (perb >= B) {
        K = B;
        while (K < 1024 && 2ll * K <= perb) K <<= 1;
      }
      if (tid == 0) {
        chunk[0] = -1;
        chunk[1] = 0;
      }
      __syncthreads();
      // phase A: short buckets; long ones are listed
      for (long long base = ds; base < de; base += gsize) {
        const long long j = base + gtid;
        const int2 d = j < de ? sc.rd_down[j] : make_int2(-1, -1);
        uint32_t lo = 0, hi = 0;
        if (d.x >= 0) {
          const uint64_t k = rd_bucket(d.x, rho);
          lo = off[k];
          hi = off[k + 1];
          if (hi - lo > (uint32_t)kRdThread) {
            // listed: blocks take the list from the front, hubs from the back
            const bool hub = (int64_t)(hi - lo) > kRdGrid;
            const unsigned slot_i = atomicAdd(hub ? hubhead : bighead, 1u);
            if ((int64_t)slot_i < sc.rd_cap) sc.rd_big[hub ? sc.rd_cap - 1 - slot_i : slot_i] = (int32_t)(j - ds);
            else raise_flag(flags, kFlagCorrupt);  // more listed entries than trail entries: impossible
            hi = lo;
          }
        }
        // as many passes as the block's longest short bucket (most are empty
        // or hold a pair or two); the trip count is block-uniform, since the
        // appends are collective
        int need = (int)(hi - lo);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) need = max(need, __shfl_xor(need, o, 64));
        if ((tid & 63) == 0) pass_max[tid >> 6] = need;
        __syncthreads();
        int passes = 0;
        for (int w = 0; w < (B >> 6); ++w) passes = max(passes, pass_max[w]);
        __syncthreads();  // pass_max is rewritten in the next iteration
        for (int it = 0; it < passes; ++it) {
          const bool have = lo + (uint32_t)it < hi;
          const int2 pr = have ? sc.rd_pairs[lo + it] : make_int2(-1, -1);
          const bool go = have && pr.x == d.x;
          if (go && d.x != d.y) st(parent + pr.y, d.y);  // a root's own children already point at it
          mine += go;
          level_put(go, make_int2(pr.y, d.y), sc.rd_down, next, K, chunk, wave_off, flags);
        }
      }
      alive = grid_sync(bar, gen, flags, spin_limit);
      if (!alive) break;
      // phase B: the listed buckets, each by one block (block b takes every
      // gridDim.x-th), then the hubs' by the whole grid.  Block 0 clears the
      // ring words one or two levels ahead (last read before this level
      // began).
      const unsigned nblk = min(ld_count(bighead), (unsigned)sc.rd_cap);
      const unsigned nhub = min(ld_count(hubhead), (unsigned)sc.rd_cap);
      if (blockIdx.x == 0 && tid == 0) {
        st_count(ring_word(sc.ctl, kBfRd + 96, level + 1), 0u);   // block-list heads of the next level
        st_count(ring_word(sc.ctl, kBfRd + 288, level + 1), 0u);  // hub-list heads of the next level
        st_count(ring_word(sc.ctl, kBfRd + 192, level + 2), 0u);  // appends of the level after
        clear_ctr(ring_ctr(sc.ctl, kBfRd, level + 2));            // reservations of the level after
      }
      // one listed bucket: the pairs of entry (v, r) in v's bucket, read by
      // the block (first = tid, step = B) or the grid (gtid, gsize)
      auto serve = [&](int64_t slot, int64_t first, int64_t step) {
        const int2 d = sc.rd_down[ds + sc.rd_big[slot]];
        const uint64_t k = rd_bucket(d.x, rho);
        const uint32_t lo = off[k], hi = off[k + 1];
        for (int64_t t0 = lo; t0 < hi; t0 += step) {
          const int64_t t = t0 + first;
          const int2 pr = t < hi ? sc.rd_pairs[t] : make_int2(-1, -1);
          const bool go = t < hi && pr.x == d.x;
          if (go && d.x != d.y) st(parent + pr.y, d.y);
          mine += go;
          level_put(go, make_int2(pr.y, d.y), sc.rd_down, next, K, chunk, wave_off, flags);
        }
      };
      for (unsigned q = blockIdx.x; q < nblk; q += gridDim.x) serve(q, tid, B);
      for (unsigned h = 0; h < nhub; ++h) serve(sc.rd_cap - 1 - h, gtid, gsize);
      __syncthreads();
      if (K > 0 && chunk[0] >= 0)
        for (long long t = chunk[1] + tid; t < K; t += B) sc.rd_down[chunk[0] + t] = make_int2(-1, -1);
      const int wm = wave_sum(mine);
      if ((tid & 63) == 0 && wm > 0) atomicAdd(realnext, (unsigned)wm);
      alive = grid_sync(bar, gen, flags, spin_limit);
      ds = de;
      const long long h = ds + (long long)ld_ctr(next.ctr);
      de = h < dcap ? h : dcap;
      real = (long long)ld_count(realnext);
      // one level per tree level: as many as the deepest traversed path
      // (id or hashed linking can build paths of any length), never more
      // levels than trail entries
      if ((long long)level > lam) {
        raise_flag(flags, kFlagCorrupt);
        alive = false;
      }
    }
  }
  // Phase II: pointer jumping over the trail (own level-0 segment + the log)
  for (int round = 0; PH2 == 0 && alive; ++round) {
    if (blockIdx.x == 0 && tid == 0) st_count(ring_word(sc.ctl, kBfFlags, round + 1), 0u);
    bool moved = false;
    for_level0(sc, [&](int32_t v) {
      if (v >= 0) moved |= jump<R>(parent, v);
    });
    for (int64_t j = gtid; j < lend; j += gsize) {
      const int32_t v = sc.log[j];
      if ((uint32_t)v < (uint32_t)n) moved |= jump<R>(parent, v);
    }
    if (__syncthreads_or(moved) && tid == 0) st_count(ring_word(sc.ctl, kBfFlags, round), 1u);
    alive = grid_sync(bar, gen, flags, spin_limit);
    if (!alive || ld_count(ring_word(sc.ctl, kBfFlags, round)) == 0u) break;
    if (round > 64) {  // deeper than any forest of 2^31 vertices after this many halvings
      raise_flag(flags, kFlagCorrupt);
      alive = false;
    }
  }
  for_level0(sc, [&](int32_t v) {
    if (v >= 0) atomicAnd(sc.visited + (v >> 5), ~(1u << (v & 31)));
  });
  for (int64_t j = gtid; j < lend; j += gsize) {
    const int32_t v = sc.log[j];
    if ((uint32_t)v < (uint32_t)n) atomicAnd(sc.visited + (v >> 5), ~(1u << (v & 31)));
  }

  // the operation itself
  if (KIND == 1) {
    // the open pairs: both ends were climbed and point at their roots
    for (int64_t i = gtid; i < count; i += gsize) {
      if (out[i] != kBfOpen) continue;
      const int2 p = items[i];
      out[i] = ldp<R>(parent + p.x) == ldp<R>(parent + p.y);
    }
  } else {
    int links = 0;
    auto settle = [&](int64_t i) {
      const int2 p = items[i];
      if (touched_bits) {
        mark_touched(touched_bits, p.x);
        mark_touched(touched_bits, p.y);
      }
      const int32_t ru = ldp<R>(parent + p.x), rv = ldp<R>(parent + p.y);  // roots before any link
      if (ru != rv) links += link(parent, ru, rv, n, flags, Ord{}) >= 0;
    };
    if (sc.open) {
      // only the items level 0 left open, from the lists of the level-0
      // blocks this block reads (the others are out of range, self-loops or
      // settled by the bits)
      const int64_t per = sc.seg0_cap >> 1;
      for (int64_t a = blockIdx.x; a < sc.seg_blocks; a += gridDim.x) {
        const uint32_t* list = sc.open + a * per;
        const int64_t nopen = sc.seg_n[2 * a + 1];
        for (int64_t k = tid; k < nopen; k += B) settle((int64_t)list[k]);
      }
    } else {
      for (int64_t i = gtid; i < count; i += gsize) {
        const int2 p = items[i];
        if (!in_range(p, n) || p.x == p.y || both_members(member, p)) continue;
        settle(i);
      }
    }
    count_links(slots, links);
  }
}

}  // namespace
}  // namespace ccdev

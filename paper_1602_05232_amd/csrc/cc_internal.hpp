// Host-side helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>

#include <vector>

#include "../../include/cc.h"

void cc_set_error(const char* fmt, ...);

#define HIP_TRY(expr)                                                               \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      cc_set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                   __LINE__);                                                       \
      return CC_EDEVICE;                                                            \
    }                                                                               \
  } while (0)

namespace cc {

// Makes `dev` current for the lifetime of the guard.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Edge and pair arrays are read 8 bytes (one pair) per load.
inline bool misaligned8(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 7u) != 0; }

inline unsigned blocks_for(int64_t items, int64_t per_block, int cap) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

struct Tuning {
  int mode = 0;             // CC_OPT_UPDATE_MODE
  int block = 256;          // CC_OPT_BLOCK
  int items = 0;            // CC_OPT_ITEMS (0 = per call)
  int query_halving = 1;    // CC_OPT_QUERY_HALVING
  int64_t compress_every = 0;  // CC_OPT_COMPRESS_EVERY
  int hook = 0;             // CC_OPT_HOOK
  int grid_cap = 4096;      // CC_OPT_GRID_CAP
  int compress_linked = 1;  // CC_OPT_COMPRESS_LINKED
  int64_t spin_limit = 1 << 24;  // CC_OPT_SPIN_LIMIT
  int find = 0;                  // CC_OPT_FIND
  int one_launch = 0;            // CC_OPT_ONE_LAUNCH (pools)
  int filter = 0;                // CC_OPT_FILTER
  int query_items = 0;           // CC_OPT_QUERY_ITEMS (0 = as CC_OPT_ITEMS)
  int split_below = 0;           // CC_OPT_SPLIT_BELOW (percent; 0 = always fused)
};

inline bool set_tuning(Tuning* t, int key, int64_t v) {
  switch (key) {
    case CC_OPT_UPDATE_MODE:
      if (v < 0 || v > 2) return false;
      t->mode = (int)v;
      return true;
    case CC_OPT_BLOCK:
      if (v < 64 || v > 1024 || v % 64) return false;
      t->block = (int)v;
      return true;
    case CC_OPT_ITEMS:
      if (v != 0 && v != 1 && v != 2 && v != 4 && v != 8) return false;
      t->items = (int)v;
      return true;
    case CC_OPT_QUERY_HALVING:
      if (v != 0 && v != 1) return false;
      t->query_halving = (int)v;
      return true;
    case CC_OPT_COMPRESS_EVERY:
      if (v < 0) return false;
      t->compress_every = v;
      return true;
    case CC_OPT_HOOK:
      if (v < 0 || v > 2) return false;
      t->hook = (int)v;
      return true;
    case CC_OPT_GRID_CAP:
      if (v < 1 || v > (1 << 20)) return false;
      t->grid_cap = (int)v;
      return true;
    case CC_OPT_COMPRESS_LINKED:
      if (v != 0 && v != 1) return false;
      t->compress_linked = (int)v;
      return true;
    case CC_OPT_SPIN_LIMIT:
      if (v < 0 || v > 0xffffffffLL) return false;
      t->spin_limit = v;
      return true;
    case CC_OPT_FIND:
      if (v < 0 || v > 2) return false;
      t->find = (int)v;
      return true;
    case CC_OPT_ONE_LAUNCH:
      if (v != 0 && v != 1) return false;
      t->one_launch = (int)v;
      return true;
    case CC_OPT_FILTER:
      if (v < 0 || v > 2) return false;
      t->filter = (int)v;
      return true;
    case CC_OPT_QUERY_ITEMS:
      if (v != 0 && v != 1 && v != 2 && v != 4 && v != 8) return false;
      t->query_items = (int)v;
      return true;
    case CC_OPT_SPLIT_BELOW:
      if (v < 0 || v > 100) return false;
      t->split_below = (int)v;
      return true;
    default:
      return false;
  }
}

inline bool get_tuning(const Tuning* t, int key, int64_t* v) {
  switch (key) {
    case CC_OPT_UPDATE_MODE: *v = t->mode; return true;
    case CC_OPT_BLOCK: *v = t->block; return true;
    case CC_OPT_ITEMS: *v = t->items; return true;
    case CC_OPT_QUERY_HALVING: *v = t->query_halving; return true;
    case CC_OPT_COMPRESS_EVERY: *v = t->compress_every; return true;
    case CC_OPT_HOOK: *v = t->hook; return true;
    case CC_OPT_GRID_CAP: *v = t->grid_cap; return true;
    case CC_OPT_COMPRESS_LINKED: *v = t->compress_linked; return true;
    case CC_OPT_SPIN_LIMIT: *v = t->spin_limit; return true;
    case CC_OPT_FIND: *v = t->find; return true;
    case CC_OPT_ONE_LAUNCH: *v = t->one_launch; return true;
    case CC_OPT_FILTER: *v = t->filter; return true;
    case CC_OPT_QUERY_ITEMS: *v = t->query_items; return true;
    case CC_OPT_SPLIT_BELOW: *v = t->split_below; return true;
    default: return false;
  }
}

// Upper bound on the blocks of a cooperative launch (every block resident
// at once): the occupancy calculator's blocks per compute unit times the
// units, less one wavefront per SIMD whenever the calculator allows 7 or
// more.  The calculator prices SGPRs against a larger register file than
// the one a grid actually gets: a residency probe (block leaders count in
// and wait, bounded, for the whole grid) with the same footprint but for
// its SGPRs found, for blocks of 256 on an idle device, that an SGPR
// allocation of 96 per wavefront fits 7 wavefronts per SIMD where the
// calculator says 8, and one of 112 fits 6 where it says 7, while 80 SGPRs
// (or 61 VGPRs) fit the calculator's 8.  Two kernels of this library hit
// it: the contracting update, 2048 blocks of 256 (1792 resident), and the
// pool's one-launch form with 4 items per thread, 1024 blocks of 512 (2.7 s
// per launch instead of 3 ms: the blocks left out ran only as the spinning
// ones were preempted).  Bounds below 7 wavefronts per SIMD come from VGPRs
// or LDS here and are kept.  Cooperative grids of this library also never
// overlap (coop_before/coop_after), and a grid that still cannot become
// resident ends at the barrier's spin limit with CC_EDEVICE.
inline int64_t coop_limit(int per_cu, int cus, int block) {
  const int wpb = (block + 63) / 64;             // wavefronts per block
  const int simd_waves = per_cu * wpb / 4;       // the calculator's wavefronts per SIMD
  int b = per_cu;
  if (simd_waves >= 7) b = (simd_waves - 1) * 4 / wpb;
  if (b > per_cu) b = per_cu;
  return (int64_t)(b > 0 ? b : 1) * cus;
}

// Cooperative launches of this library never overlap on a device.  Each
// sizes its grid to nearly fill the device and waits at device-wide barriers
// until every block is resident, so two of them running at once (different
// graphs or pool runs on different streams) could each hold compute units
// the other waits for.  coop_before(stream) makes `stream` wait (on the
// device, without blocking the host) for the last cooperative launch issued
// on another stream of the current device; coop_after(stream) records the
// launch just issued on `stream` as the last one.  Thread safe.
int coop_before(hipStream_t stream);
int coop_after(hipStream_t stream);

// Items per thread for a launch over m items: the requested value, or with
// 0 the largest of 8, 4, 2, 1 that still gives at least 2048 blocks.
inline int pick_items(int requested, int64_t m, int block) {
  if (requested > 0) return requested;
  int it = 8;
  while (it > 1 && m < (int64_t)block * it * 2048) it >>= 1;
  return it;
}

inline uint32_t fmix32_host(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}

// A parent image is a valid forest under the linking order when every
// pointer stays in range and goes from lower to strictly higher priority
// (then no cycle is possible).  Under union by rank (hook 2) a root's word
// carries its rank in the bits above kRankShift and the order is not
// recoverable from the image, so every path is walked instead (each node is
// visited once; a walk that meets itself is a cycle).  Counts the roots.
inline bool check_forest(const int32_t* p, int64_t n, int hook, int64_t* roots) {
  if (hook == 2) {
    constexpr int32_t mask = (1 << 27) - 1;
    std::vector<uint8_t> state((size_t)n, 0);  // 0 new, 1 on the current walk, 2 done
    int64_t r = 0;
    for (int64_t v = 0; v < n; ++v) {
      int64_t x = v;
      while (state[(size_t)x] == 0) {
        state[(size_t)x] = 1;
        const int32_t w = p[x];  // a high rank sets the sign bit
        const int32_t q = w & mask;
        if (q >= n) return false;
        if (q == x) {
          ++r;
          break;
        }
        if (w != q) return false;  // only roots carry rank bits
        x = q;
      }
      if (state[(size_t)x] == 1 && (p[x] & mask) != x) return false;  // met its own walk
      for (int64_t y = v; state[(size_t)y] == 1;) {
        state[(size_t)y] = 2;
        const int32_t q = p[y] & mask;
        if (q == y) break;
        y = q;
      }
    }
    *roots = r;
    return true;
  }
  int64_t r = 0;
  for (int64_t v = 0; v < n; ++v) {
    const int32_t q = p[v];
    if (q < 0 || q >= n) return false;
    if (q == v) {
      ++r;
      continue;
    }
    const bool ok = hook == 1 ? fmix32_host((uint32_t)q) < fmix32_host((uint32_t)v) : q < v;
    if (!ok) return false;
  }
  *roots = r;
  return true;
}

}  // namespace cc

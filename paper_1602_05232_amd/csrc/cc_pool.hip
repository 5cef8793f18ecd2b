// C ABI of the many-graph pool (include/cc_pool.h).

// Path-shortening stores at workgroup scope: Bulk-Find, whose response
// distributor needs those stores visible device-wide by the next launch, is
// never run on a pool's graphs, and the pool's finds tolerate a late store
// (an older ancestor is still an ancestor).  Measured on the 1024-graph
// workload: 2.63 -> 2.39 ms per minibatch round against agent scope.
#define CC_PATH_STORE_SCOPE __HIP_MEMORY_SCOPE_WORKGROUP

#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <vector>

#include "../../include/cc_pool.h"
#include "cc_internal.hpp"
#include "cc_pool_kernels.hpp"

using namespace ccdev;
using cc::blocks_for;
using cc::DeviceGuard;

namespace {

constexpr int kRing = 4;  // descriptor staging slots in flight

struct PoolGraph {
  int64_t base = 0, n = 0;
  bool used = false;
};

// One run in flight: its descriptors, the list of roots its updates linked
// (compressed after each round), and the device-wide barrier of its
// one-launch form.  A slot is reused only after its run has completed, so
// runs on different streams never share a list or a barrier.
struct RingSlot {
  OpDesc* host = nullptr;  // pinned staging
  OpDesc* dev = nullptr;
  int64_t cap = 0;
  int2* hooked = nullptr;     // capacity entries (graph base, local id), allocated on first use
  unsigned* ctl = nullptr;    // [0] hooked count, [1] finished blocks
  int32_t* meta_host = nullptr;  // one-launch form: round starts, then round tiles
  int32_t* meta_dev = nullptr;
  int64_t meta_cap = 0;
  unsigned* bar = nullptr;    // kBarWords, allocated on the first one-launch run
  hipEvent_t done = nullptr;
  bool pending = false;
};

}  // namespace

struct cc_pool {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t capacity = 0;
  int32_t max_graphs = 0;
  int32_t* arena = nullptr;
  unsigned long long* glinks = nullptr;  // max_graphs * kPoolLinkStride
  int* flags = nullptr;
  std::vector<PoolGraph> graphs;
  std::map<int64_t, int64_t> gaps;  // base -> length of each free range
  int32_t* staging = nullptr;       // device image buffer for save / load
  int64_t staging_cap = 0;
  unsigned long long* check = nullptr;  // [0] bad entries, [1] roots (image check)
  int2* table = nullptr;                // (base, n) of the graphs in use, for cc_pool_reset_all
  std::vector<int2> table_host;
  bool table_stale = true;              // graphs added or removed since the table was uploaded
  uint32_t* member = nullptr;           // membership filter: one bit per arena slot (+1 word)
  int32_t* anchors = nullptr;           // membership filter: anchor vertex per graph handle, -1 for none,
                                        // then (aroot) the anchor's root at the last refresh, -1 for no bits
  std::vector<int64_t> unrefreshed;     // membership filter: update edges since the graph's bits were renewed
  RingSlot ring[kRing];
  int ring_next = 0;
  cc::Tuning tune;
};

namespace {

bool valid_graph(const cc_pool* p, int32_t id) {
  return p && id >= 0 && id < p->max_graphs && p->graphs[(size_t)id].used;
}

int64_t take_gap(cc_pool* p, int64_t n) {
  for (auto it = p->gaps.begin(); it != p->gaps.end(); ++it) {
    if (it->second >= n) {
      const int64_t base = it->first, len = it->second;
      p->gaps.erase(it);
      if (len > n) p->gaps[base + n] = len - n;
      return base;
    }
  }
  return -1;
}

void give_gap(cc_pool* p, int64_t base, int64_t n) {
  auto it = p->gaps.emplace(base, n).first;
  auto nx = std::next(it);
  if (nx != p->gaps.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    p->gaps.erase(nx);
  }
  if (it != p->gaps.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      p->gaps.erase(it);
    }
  }
}

int reserve_slot(cc_pool* p, int64_t count, bool record, bool one_launch, RingSlot** out) {
  RingSlot* s = &p->ring[p->ring_next];
  p->ring_next = (p->ring_next + 1) % kRing;
  if (s->pending) {
    HIP_TRY(hipEventSynchronize(s->done));
    s->pending = false;
  }
  if (s->cap < count) {
    if (s->host) (void)hipHostFree(s->host);
    if (s->dev) (void)hipFree(s->dev);
    s->host = nullptr;
    s->dev = nullptr;
    s->cap = 0;
    const int64_t cap = std::max<int64_t>(count, 1024);
    if (hipHostMalloc((void**)&s->host, (size_t)cap * sizeof(OpDesc), hipHostMallocDefault) != hipSuccess ||
        hipMalloc((void**)&s->dev, (size_t)cap * sizeof(OpDesc)) != hipSuccess) {
      cc_set_error("cc_pool_run: descriptor staging allocation failed");
      return CC_ENOMEM;
    }
    s->cap = cap;
  }
  if (record && !s->hooked) {
    if (hipMalloc((void**)&s->hooked, (size_t)p->capacity * sizeof(int2)) != hipSuccess ||
        hipMalloc((void**)&s->ctl, 64) != hipSuccess) {
      cc_set_error("cc_pool_run: hooked-list allocation failed");
      return CC_ENOMEM;
    }
    HIP_TRY(hipMemsetAsync(s->ctl, 0, 64, p->stream));
  }
  if (one_launch && !s->bar && hipMalloc((void**)&s->bar, kBarWords * sizeof(unsigned)) != hipSuccess) {
    s->bar = nullptr;
    cc_set_error("cc_pool_run: barrier allocation failed");
    return CC_ENOMEM;
  }
  *out = s;
  return CC_OK;
}

int reserve_meta(RingSlot* s, int64_t words) {
  if (s->meta_cap >= words) return CC_OK;
  if (s->meta_host) (void)hipHostFree(s->meta_host);
  if (s->meta_dev) (void)hipFree(s->meta_dev);
  s->meta_host = nullptr;
  s->meta_dev = nullptr;
  s->meta_cap = 0;
  const int64_t cap = std::max<int64_t>(words, 256);
  if (hipHostMalloc((void**)&s->meta_host, (size_t)cap * 4, hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void**)&s->meta_dev, (size_t)cap * 4) != hipSuccess) {
    cc_set_error("cc_pool_run: round table allocation failed");
    return CC_ENOMEM;
  }
  s->meta_cap = cap;
  return CC_OK;
}

template <int ITEMS, int HOOK, bool HALVE, bool FILT>
int launch_rounds_t(cc_pool* p, const RingSlot* s, int rounds, uint32_t max_tiles, const OpDesc* fops) {
  const int B = p->tune.block;
  int per_cu = 0, cus = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_pool_rounds<ITEMS, HOOK, HALVE, FILT>, B, 0));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device));
  int64_t grid = std::min<int64_t>(std::min<int64_t>(max_tiles, cc::coop_limit(per_cu, cus, B)), p->tune.grid_cap);
  grid = std::max<int64_t>(grid, 1);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, p->stream, s->bar, kBarWords);
  HIP_TRY(hipGetLastError());
  const OpDesc* ops = s->dev;
  const int32_t* rstart = s->meta_dev;
  const uint32_t* rtiles = reinterpret_cast<const uint32_t*>(s->meta_dev + rounds + 1);
  int32_t* arena = p->arena;
  unsigned long long* glinks = p->glinks;
  int* flags = p->flags;
  unsigned* bar = s->bar;
  unsigned spin = (unsigned)p->tune.spin_limit;
  uint32_t* member = p->member;
  int32_t* anchors = p->anchors;
  int32_t* aroot = p->anchors ? p->anchors + p->max_graphs : nullptr;
  // refresh table after the round table: starts (rounds + 1), then tiles
  const int32_t* fstart = s->meta_dev + 2 * rounds + 1;
  const uint32_t* ftiles = reinterpret_cast<const uint32_t*>(s->meta_dev + 3 * rounds + 2);
  void* args[] = {&ops,    &rstart,  &rtiles, &rounds, &arena, &glinks, &flags,  &bar,
                  &spin,   &member,  &anchors, &aroot, &fops,  &fstart, &ftiles};
  if (const int crc = cc::coop_before(p->stream)) return crc;
  HIP_TRY(hipLaunchCooperativeKernel((const void*)k_pool_rounds<ITEMS, HOOK, HALVE, FILT>, dim3((unsigned)grid),
                                     dim3(B), args, 0, p->stream));
  if (const int crc = cc::coop_after(p->stream)) return crc;
  return CC_OK;
}

template <int ITEMS, int HOOK, bool FILT>
int launch_rounds_f(cc_pool* p, const RingSlot* s, int rounds, uint32_t max_tiles, const OpDesc* fops) {
  return p->tune.query_halving ? launch_rounds_t<ITEMS, HOOK, true, FILT>(p, s, rounds, max_tiles, fops)
                               : launch_rounds_t<ITEMS, HOOK, false, FILT>(p, s, rounds, max_tiles, fops);
}

template <int ITEMS, int HOOK>
int launch_rounds_h(cc_pool* p, const RingSlot* s, int rounds, uint32_t max_tiles, const OpDesc* fops) {
  return p->tune.filter && p->member ? launch_rounds_f<ITEMS, HOOK, true>(p, s, rounds, max_tiles, fops)
                                     : launch_rounds_f<ITEMS, HOOK, false>(p, s, rounds, max_tiles, fops);
}

template <int ITEMS>
int launch_rounds_i(cc_pool* p, const RingSlot* s, int rounds, uint32_t max_tiles, const OpDesc* fops) {
  switch (p->tune.hook) {
    case 1: return launch_rounds_h<ITEMS, 1>(p, s, rounds, max_tiles, fops);
    case 2: return launch_rounds_h<ITEMS, 2>(p, s, rounds, max_tiles, fops);
    default: return launch_rounds_h<ITEMS, 0>(p, s, rounds, max_tiles, fops);
  }
}

// fops: the run's refresh descriptors (membership filter)
int launch_rounds(cc_pool* p, const RingSlot* s, int items, int rounds, uint32_t max_tiles, const OpDesc* fops) {
  switch (items) {
    case 1: return launch_rounds_i<1>(p, s, rounds, max_tiles, fops);
    case 2: return launch_rounds_i<2>(p, s, rounds, max_tiles, fops);
    case 8: return launch_rounds_i<8>(p, s, rounds, max_tiles, fops);
    default: return launch_rounds_i<4>(p, s, rounds, max_tiles, fops);
  }
}

template <int ITEMS, int HOOK, bool RECORD, bool FILT>
void launch_phase_t(cc_pool* p, const RingSlot* s, const OpDesc* d, int nops, uint32_t ntiles) {
  const int B = p->tune.block;
  const unsigned grid = (unsigned)std::min<int64_t>(ntiles, p->tune.grid_cap);
  const int32_t* aroot = p->anchors ? p->anchors + p->max_graphs : nullptr;
  if (p->tune.query_halving)
    hipLaunchKernelGGL((k_pool_phase<ITEMS, HOOK, RECORD, true, FILT>), dim3(grid), dim3(B), 0, p->stream, d, nops,
                       ntiles, p->arena, p->glinks, p->flags, s->hooked, s->ctl, p->member, aroot);
  else
    hipLaunchKernelGGL((k_pool_phase<ITEMS, HOOK, RECORD, false, FILT>), dim3(grid), dim3(B), 0, p->stream, d, nops,
                       ntiles, p->arena, p->glinks, p->flags, s->hooked, s->ctl, p->member, aroot);
}

template <int ITEMS, int HOOK, bool FILT>
void launch_phase_f(cc_pool* p, const RingSlot* s, const OpDesc* d, int nops, uint32_t ntiles, bool record) {
  if (record) launch_phase_t<ITEMS, HOOK, true, FILT>(p, s, d, nops, ntiles);
  else launch_phase_t<ITEMS, HOOK, false, FILT>(p, s, d, nops, ntiles);
}

template <int ITEMS, int HOOK>
void launch_phase_h(cc_pool* p, const RingSlot* s, const OpDesc* d, int nops, uint32_t ntiles, bool record) {
  if (p->tune.filter && p->member) launch_phase_f<ITEMS, HOOK, true>(p, s, d, nops, ntiles, record);
  else launch_phase_f<ITEMS, HOOK, false>(p, s, d, nops, ntiles, record);
}

// Membership filter: clear the bits of arena slots [base, base + n) and the
// anchors of handles [g0, g1) (no-op while the filter is off; turning it on
// clears everything).
int filter_clear(cc_pool* p, int64_t base, int64_t n, int32_t g0, int32_t g1) {
  if (!p->tune.filter || !p->member) return CC_OK;
  const int64_t work = std::max<int64_t>((n + 31) / 32 + 1, g1 - g0);
  hipLaunchKernelGGL(k_pool_filter_clear, dim3(blocks_for(work, 256, 4096)), dim3(256), 0, p->stream, p->member,
                     base, n, p->anchors, p->anchors + p->max_graphs, g0, g1);
  HIP_TRY(hipGetLastError());
  for (int32_t g = g0; g < g1; ++g) p->unrefreshed[(size_t)g] = 0;
  return CC_OK;
}

constexpr int kRefreshBlock = 256;  // bitmap words per refresh tile

// Before an update round: anchor roots, then the refresh pass, for the
// graphs listed in d (nops descriptors with word-tile offsets).
void filter_refresh(cc_pool* p, const OpDesc* d, int nops, uint32_t ntiles) {
  int32_t* aroot = p->anchors + p->max_graphs;
  const unsigned tiles = (unsigned)std::min<int64_t>(ntiles, 8192);
  if (p->tune.hook == 2) {
    hipLaunchKernelGGL(k_pool_filter_roots<true>, dim3((nops + 255) / 256), dim3(256), 0, p->stream, d, nops,
                       p->arena, p->anchors, aroot, p->flags);
    hipLaunchKernelGGL(k_pool_filter_refresh<true>, dim3(tiles), dim3(kRefreshBlock), 0, p->stream, d, nops, ntiles,
                       p->arena, p->member, aroot);
  } else {
    hipLaunchKernelGGL(k_pool_filter_roots<false>, dim3((nops + 255) / 256), dim3(256), 0, p->stream, d, nops,
                       p->arena, p->anchors, aroot, p->flags);
    hipLaunchKernelGGL(k_pool_filter_refresh<false>, dim3(tiles), dim3(kRefreshBlock), 0, p->stream, d, nops, ntiles,
                       p->arena, p->member, aroot);
  }
}

template <int ITEMS>
void launch_phase_i(cc_pool* p, const RingSlot* s, const OpDesc* d, int nops, uint32_t ntiles, bool record) {
  switch (p->tune.hook) {
    case 1: launch_phase_h<ITEMS, 1>(p, s, d, nops, ntiles, record); break;
    case 2: launch_phase_h<ITEMS, 2>(p, s, d, nops, ntiles, record); break;
    default: launch_phase_h<ITEMS, 0>(p, s, d, nops, ntiles, record); break;
  }
}

void launch_phase(cc_pool* p, const RingSlot* s, int items, const OpDesc* d, int nops, uint32_t ntiles,
                  bool record) {
  switch (items) {
    case 1: launch_phase_i<1>(p, s, d, nops, ntiles, record); break;
    case 2: launch_phase_i<2>(p, s, d, nops, ntiles, record); break;
    case 8: launch_phase_i<8>(p, s, d, nops, ntiles, record); break;
    default: launch_phase_i<4>(p, s, d, nops, ntiles, record); break;
  }
}

}  // namespace

extern "C" cc_pool* cc_pool_create(int64_t capacity, int32_t max_graphs) {
  if (capacity < 1 || capacity > 0x7fffffffLL || max_graphs < 1 || max_graphs > (1 << 24)) {
    cc_set_error("cc_pool_create: capacity %lld / max_graphs %d out of range", (long long)capacity, max_graphs);
    return nullptr;
  }
  cc_pool* p = new (std::nothrow) cc_pool();
  if (!p) return nullptr;
  p->capacity = capacity;
  p->max_graphs = max_graphs;
  p->graphs.resize((size_t)max_graphs);
  p->unrefreshed.assign((size_t)max_graphs, 0);
  p->gaps[0] = capacity;
  auto fail = [&](const char* what) -> cc_pool* {
    cc_set_error("cc_pool_create: %s failed", what);
    (void)hipFree(p->arena);
    (void)hipFree(p->glinks);
    (void)hipFree(p->flags);
    (void)hipFree(p->table);
    delete p;
    return nullptr;
  };
  if (hipGetDevice(&p->device) != hipSuccess) return fail("hipGetDevice");
  if (hipMalloc(&p->arena, (size_t)capacity * 4) != hipSuccess) return fail("arena");
  if (hipMalloc(&p->glinks, (size_t)max_graphs * kPoolLinkStride * 8) != hipSuccess) return fail("links");
  if (hipMalloc(&p->flags, 64) != hipSuccess) return fail("flags");
  if (hipMalloc(&p->table, (size_t)max_graphs * sizeof(int2)) != hipSuccess) return fail("table");
  if (hipMemsetAsync(p->flags, 0, 64, p->stream) != hipSuccess) return fail("memset");
  if (hipMemsetAsync(p->glinks, 0, (size_t)max_graphs * kPoolLinkStride * 8, p->stream) != hipSuccess)
    return fail("memset");
  for (auto& s : p->ring)
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess) return fail("event");
  if (hipStreamSynchronize(p->stream) != hipSuccess) return fail("sync");
  return p;
}

extern "C" int cc_pool_destroy(cc_pool* p) {
  if (!p) return CC_EINVAL;
  DeviceGuard dg(p->device);
  (void)hipStreamSynchronize(p->stream);
  for (auto& s : p->ring) {
    if (s.done) (void)hipEventSynchronize(s.done);
    if (s.host) (void)hipHostFree(s.host);
    if (s.dev) (void)hipFree(s.dev);
    if (s.hooked) (void)hipFree(s.hooked);
    if (s.ctl) (void)hipFree(s.ctl);
    if (s.meta_host) (void)hipHostFree(s.meta_host);
    if (s.meta_dev) (void)hipFree(s.meta_dev);
    if (s.bar) (void)hipFree(s.bar);
    if (s.done) (void)hipEventDestroy(s.done);
  }
  (void)hipFree(p->arena);
  (void)hipFree(p->glinks);
  (void)hipFree(p->flags);
  (void)hipFree(p->staging);
  (void)hipFree(p->check);
  (void)hipFree(p->table);
  (void)hipFree(p->member);
  (void)hipFree(p->anchors);
  delete p;
  return CC_OK;
}

extern "C" int cc_pool_set_stream(cc_pool* p, void* stream) {
  if (!p) return CC_EINVAL;
  p->stream = (hipStream_t)stream;
  return CC_OK;
}

extern "C" int cc_pool_set_option(cc_pool* p, int key, int64_t value) {
  if (!p) return CC_EINVAL;
  if (key == CC_OPT_UPDATE_MODE || key == CC_OPT_COMPRESS_EVERY || key == CC_OPT_FIND || key == CC_OPT_QUERY_ITEMS ||
      key == CC_OPT_SPLIT_BELOW) {
    cc_set_error("cc_pool_set_option: option %d does not apply to pools", key);
    return CC_EINVAL;
  }
  if (key == CC_OPT_HOOK) {
    for (const auto& g : p->graphs)
      if (g.used) {
        cc_set_error("cc_pool_set_option: the linking order is fixed once a graph exists");
        return CC_EINVAL;
      }
  }
  if (key == CC_OPT_FILTER) {
    if (value != 0 && value != 1) {
      cc_set_error("cc_pool_set_option: the pool's filter is 0 (off) or 1 (on), not %lld", (long long)value);
      return CC_EINVAL;
    }
    if (value == 1 && !p->tune.filter) {
      DeviceGuard dg(p->device);
      const int64_t words = p->capacity / 32 + 1;
      if (!p->member && hipMalloc((void**)&p->member, (size_t)words * 4) != hipSuccess) {
        p->member = nullptr;
        cc_set_error("cc_pool_set_option: membership bitmap allocation failed");
        return CC_ENOMEM;
      }
      if (!p->anchors && hipMalloc((void**)&p->anchors, (size_t)p->max_graphs * 8) != hipSuccess) {
        p->anchors = nullptr;
        cc_set_error("cc_pool_set_option: anchor table allocation failed");
        return CC_ENOMEM;
      }
      p->tune.filter = 1;
      // bits kept while the filter was off may describe forests since reset
      if (const int rc = filter_clear(p, 0, p->capacity, 0, p->max_graphs)) return rc;
      for (int32_t g = 0; g < p->max_graphs; ++g)  // a forest of unknown age: renew at its next update
        p->unrefreshed[(size_t)g] = p->graphs[(size_t)g].used ? p->graphs[(size_t)g].n : 0;
      return CC_OK;
    }
    p->tune.filter = (int)value;
    return CC_OK;
  }
  if (!cc::set_tuning(&p->tune, key, value)) {
    cc_set_error("cc_pool_set_option: key %d value %lld rejected", key, (long long)value);
    return CC_EINVAL;
  }
  return CC_OK;
}

extern "C" int cc_pool_add(cc_pool* p, int64_t n, int32_t* id) {
  if (!p || !id || n < 1) return CC_EINVAL;
  if (p->tune.hook == 2 && n > (int64_t)kIdMask + 1) {
    cc_set_error("cc_pool_add: union by rank needs graphs of at most 2^%d vertices", kRankShift);
    return CC_EINVAL;
  }
  DeviceGuard dg(p->device);
  int32_t slot = -1;
  for (int32_t i = 0; i < p->max_graphs; ++i)
    if (!p->graphs[(size_t)i].used) {
      slot = i;
      break;
    }
  if (slot < 0) {
    cc_set_error("cc_pool_add: all %d graph handles in use", p->max_graphs);
    return CC_ENOMEM;
  }
  const int64_t base = take_gap(p, n);
  if (base < 0) {
    cc_set_error("cc_pool_add: no free range of %lld vertices", (long long)n);
    return CC_ENOMEM;
  }
  PoolGraph& g = p->graphs[(size_t)slot];
  g.base = base;
  g.n = n;
  g.used = true;
  p->table_stale = true;
  hipLaunchKernelGGL(k_init_range, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, p->stream, p->arena,
                     (int32_t)base, (int32_t)n);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, p->stream, p->glinks + (size_t)slot * kPoolLinkStride, 1);
  HIP_TRY(hipGetLastError());
  if (const int rc = filter_clear(p, base, n, slot, slot + 1)) return rc;
  *id = slot;
  return CC_OK;
}

extern "C" int cc_pool_remove(cc_pool* p, int32_t id) {
  if (!valid_graph(p, id)) return CC_EINVAL;
  PoolGraph& g = p->graphs[(size_t)id];
  give_gap(p, g.base, g.n);
  g = PoolGraph();
  p->table_stale = true;
  return CC_OK;
}

extern "C" int cc_pool_reset(cc_pool* p, int32_t id) {
  if (!valid_graph(p, id)) return CC_EINVAL;
  DeviceGuard dg(p->device);
  const PoolGraph& g = p->graphs[(size_t)id];
  hipLaunchKernelGGL(k_init_range, dim3(blocks_for(g.n, 256, 4096)), dim3(256), 0, p->stream, p->arena,
                     (int32_t)g.base, (int32_t)g.n);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, p->stream, p->glinks + (size_t)id * kPoolLinkStride, 1);
  HIP_TRY(hipGetLastError());
  return filter_clear(p, g.base, g.n, id, id + 1);
}

extern "C" int cc_pool_reset_all(cc_pool* p) {
  if (!p) return CC_EINVAL;
  DeviceGuard dg(p->device);
  std::vector<int2>& t = p->table_host;
  if (p->table_stale) {
    t.clear();
    for (const auto& g : p->graphs)
      if (g.used) t.push_back(make_int2((int32_t)g.base, (int32_t)g.n));
    std::sort(t.begin(), t.end(), [](const int2& a, const int2& b) { return a.x < b.x; });
    if (!t.empty()) {
      // uploaded only when the set of graphs changed; waits so that the
      // host table may be rebuilt next time
      HIP_TRY(hipMemcpyAsync(p->table, t.data(), t.size() * sizeof(int2), hipMemcpyHostToDevice, p->stream));
      HIP_TRY(hipStreamSynchronize(p->stream));
    }
    p->table_stale = false;
  }
  if (!t.empty()) {
    hipLaunchKernelGGL(k_pool_init_all, dim3(blocks_for(p->capacity, 256, 4096)), dim3(256), 0, p->stream, p->arena,
                       p->capacity, p->table, (int)t.size());
  }
  hipLaunchKernelGGL(k_zero_u64, dim3(64), dim3(256), 0, p->stream, p->glinks, p->max_graphs * kPoolLinkStride);
  HIP_TRY(hipGetLastError());
  return filter_clear(p, 0, p->capacity, 0, p->max_graphs);
}

extern "C" int64_t cc_pool_graph_vertices(const cc_pool* p, int32_t id) {
  return valid_graph(p, id) ? p->graphs[(size_t)id].n : 0;
}

extern "C" int64_t cc_pool_free_vertices(const cc_pool* p) {
  if (!p) return 0;
  int64_t s = 0;
  for (const auto& kv : p->gaps) s += kv.second;
  return s;
}

extern "C" int64_t cc_pool_graph_base(const cc_pool* p, int32_t id) {
  return valid_graph(p, id) ? p->graphs[(size_t)id].base : -1;
}

extern "C" int32_t cc_pool_gaps(const cc_pool* p, int64_t* bases, int64_t* lengths, int32_t max) {
  if (!p) return 0;
  int32_t i = 0;
  for (const auto& kv : p->gaps) {
    if (i < max && bases && lengths) {
      bases[i] = kv.first;
      lengths[i] = kv.second;
    }
    ++i;
  }
  return i;
}

extern "C" int64_t cc_pool_largest_gap(const cc_pool* p) {
  if (!p) return 0;
  int64_t s = 0;
  for (const auto& kv : p->gaps) s = std::max(s, kv.second);
  return s;
}

extern "C" int cc_pool_run(cc_pool* p, const cc_op* ops, int32_t num_ops) {
  if (!p || num_ops < 0 || (num_ops > 0 && !ops)) return CC_EINVAL;
  // validate everything first
  std::vector<int32_t> round(num_ops > 0 ? (size_t)num_ops : 1);
  std::vector<int32_t> seen((size_t)p->max_graphs, 0);
  int32_t rounds = 0;
  int64_t live = 0;
  for (int32_t i = 0; i < num_ops; ++i) {
    const cc_op& o = ops[i];
    if (!valid_graph(p, o.graph) || (o.kind != 0 && o.kind != 1) || o.count < 0 ||
        (o.count > 0 && (!o.items || cc::misaligned8(o.items) || (o.kind == 1 && !o.out)))) {
      cc_set_error("cc_pool_run: operation %d is invalid", i);
      return CC_EINVAL;
    }
    round[(size_t)i] = seen[(size_t)o.graph]++;
    rounds = std::max(rounds, round[(size_t)i] + 1);
    live += o.count > 0;
  }
  if (live == 0) return CC_OK;
  DeviceGuard dg(p->device);
  bool any_update = false;
  for (int32_t i = 0; i < num_ops; ++i) any_update |= ops[i].kind == 0 && ops[i].count > 0;
  const bool one_launch = p->tune.one_launch != 0;
  const bool filt = p->tune.filter != 0 && p->member != nullptr;
  RingSlot* slot = nullptr;
  int rc = reserve_slot(p, filt ? 2 * live : live, any_update && p->tune.compress_linked && !one_launch, one_launch,
                        &slot);
  if (rc != CC_OK) return rc;
  const int B = p->tune.block;
  // lay the descriptors out round by round; each round gets its own items per thread
  std::vector<int64_t> rstart((size_t)rounds + 1, 0), ritems((size_t)rounds, 0), rcount((size_t)rounds, 0);
  std::vector<bool> rupd((size_t)rounds, false);
  for (int32_t i = 0; i < num_ops; ++i) {
    if (ops[i].count == 0) continue;
    const int r = round[(size_t)i];
    rcount[(size_t)r]++;
    ritems[(size_t)r] += ops[i].count;
    if (ops[i].kind == 0) rupd[(size_t)r] = true;
  }
  for (int r = 0; r < rounds; ++r) rstart[(size_t)r + 1] = rstart[(size_t)r] + rcount[(size_t)r];
  std::vector<int64_t> fill(rstart.begin(), rstart.end() - 1);
  std::vector<int> ritem_per_thread((size_t)rounds);
  std::vector<uint32_t> rtiles((size_t)rounds, 0);
  int64_t max_round_items = 0;
  for (int r = 0; r < rounds; ++r) max_round_items = std::max(max_round_items, ritems[(size_t)r]);
  for (int r = 0; r < rounds; ++r)
    ritem_per_thread[(size_t)r] = cc::pick_items(p->tune.items, one_launch ? max_round_items : ritems[(size_t)r], B);
  for (int32_t i = 0; i < num_ops; ++i) {
    const cc_op& o = ops[i];
    if (o.count == 0) continue;
    const int r = round[(size_t)i];
    const PoolGraph& g = p->graphs[(size_t)o.graph];
    const int64_t tile = (int64_t)B * ritem_per_thread[(size_t)r];
    OpDesc& d = slot->host[fill[(size_t)r]++];
    d.items = reinterpret_cast<const int2*>(o.items);
    d.out = o.out;
    d.count = o.count;
    d.base = (int32_t)g.base;
    d.n = (int32_t)g.n;
    d.kind = o.kind;
    d.graph = o.graph;
    d.tile0 = rtiles[(size_t)r];
    d.pad = 0;
    const int64_t nt = (o.count + tile - 1) / tile;
    if ((int64_t)rtiles[(size_t)r] + nt > 0xffffffffLL) {
      cc_set_error("cc_pool_run: too many tiles in one round");
      return CC_EINVAL;
    }
    rtiles[(size_t)r] += (uint32_t)nt;
  }
  // membership filter: refresh descriptors (after the `live` round
  // descriptors) for the update operations of each round whose graph has
  // taken at least n / 8 edges since its bits were last renewed (the
  // one-launch form renews inside its launch)
  std::vector<int64_t> fstart((size_t)rounds, live), fcount((size_t)rounds, 0);
  std::vector<uint32_t> ftiles((size_t)rounds, 0);
  int64_t nref = 0;
  if (filt) {
    const int64_t words_per_tile = one_launch ? B : kRefreshBlock;  // the refresh's block width
    for (int r = 0; r < rounds; ++r) {
      fstart[(size_t)r] = live + nref;
      for (int64_t i = rstart[(size_t)r]; i < rstart[(size_t)r + 1]; ++i) {
        const OpDesc& d = slot->host[i];
        // renew once the graph has taken n / 8 edges since: the pass costs
        // O(n), and a stale bit is only a missed shortcut
        int64_t& since = p->unrefreshed[(size_t)d.graph];
        if (d.kind != 0 || since == 0 || 8 * since < (int64_t)d.n) continue;
        since = 0;
        OpDesc& f = slot->host[live + nref++];
        f = d;
        f.tile0 = ftiles[(size_t)r];
        const int64_t words = (((int64_t)d.base + d.n - 1) >> 5) - ((int64_t)d.base >> 5) + 1;
        ftiles[(size_t)r] += (uint32_t)((words + words_per_tile - 1) / words_per_tile);  // at most 2^26 in all
        fcount[(size_t)r]++;
      }
      for (int64_t i = rstart[(size_t)r]; i < rstart[(size_t)r + 1]; ++i)
        if (slot->host[i].kind == 0) p->unrefreshed[(size_t)slot->host[i].graph] += slot->host[i].count;
    }
  }
  HIP_TRY(hipMemcpyAsync(slot->dev, slot->host, (size_t)(live + nref) * sizeof(OpDesc), hipMemcpyHostToDevice,
                         p->stream));
  if (one_launch) {
    // compact the non-empty rounds into the round table: starts, then tiles
    std::vector<int> used;
    for (int r = 0; r < rounds; ++r)
      if (rcount[(size_t)r] > 0) used.push_back(r);
    const int nr = (int)used.size();
    rc = reserve_meta(slot, 4 * (int64_t)nr + 2);
    if (rc != CC_OK) return rc;
    uint32_t max_tiles = 1;
    // round table: starts (nr + 1), tiles (nr); then the refresh table:
    // starts relative to the first refresh descriptor (nr + 1), tiles (nr)
    int32_t* fs = slot->meta_host + 2 * nr + 1;
    int32_t* ft = slot->meta_host + 3 * nr + 2;
    for (int k = 0; k < nr; ++k) {
      const size_t r = (size_t)used[(size_t)k];
      slot->meta_host[k] = (int32_t)rstart[r];
      slot->meta_host[nr + 1 + k] = (int32_t)rtiles[r];
      max_tiles = std::max(max_tiles, rtiles[r]);
      fs[k] = (int32_t)(fstart[r] - live);
      ft[k] = (int32_t)ftiles[r];
      max_tiles = std::max(max_tiles, ftiles[r]);
    }
    slot->meta_host[nr] = (int32_t)(rstart[(size_t)used[(size_t)nr - 1]] + rcount[(size_t)used[(size_t)nr - 1]]);
    fs[nr] = (int32_t)(fstart[(size_t)used[(size_t)nr - 1]] - live + fcount[(size_t)used[(size_t)nr - 1]]);
    HIP_TRY(hipMemcpyAsync(slot->meta_dev, slot->meta_host, (size_t)(4 * nr + 2) * 4, hipMemcpyHostToDevice,
                           p->stream));
    rc = launch_rounds(p, slot, ritem_per_thread[0], nr, max_tiles, slot->dev + live);
    if (rc != CC_OK) return rc;
    HIP_TRY(hipEventRecord(slot->done, p->stream));
    slot->pending = true;
    return CC_OK;
  }
  for (int r = 0; r < rounds; ++r) {
    if (rcount[(size_t)r] == 0) continue;
    if (fcount[(size_t)r] > 0)
      filter_refresh(p, slot->dev + fstart[(size_t)r], (int)fcount[(size_t)r], ftiles[(size_t)r]);
    const bool record = rupd[(size_t)r] && p->tune.compress_linked;
    launch_phase(p, slot, ritem_per_thread[(size_t)r], slot->dev + rstart[(size_t)r], (int)rcount[(size_t)r],
                 rtiles[(size_t)r], record);
    if (record) {
      const int32_t cap = (int32_t)std::min<int64_t>(p->capacity, 0x7fffffff);
      if (p->tune.hook == 2)
        hipLaunchKernelGGL(k_pool_compress_hooked<true>, dim3(1024), dim3(256), 0, p->stream, p->arena,
                           slot->hooked, slot->ctl, cap, p->flags);
      else
        hipLaunchKernelGGL(k_pool_compress_hooked<false>, dim3(1024), dim3(256), 0, p->stream, p->arena,
                           slot->hooked, slot->ctl, cap, p->flags);
    }
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventRecord(slot->done, p->stream));
  slot->pending = true;
  return CC_OK;
}

extern "C" int cc_pool_labels(cc_pool* p, int32_t id, int32_t* out) {
  if (!valid_graph(p, id) || !out) return CC_EINVAL;
  DeviceGuard dg(p->device);
  const PoolGraph& g = p->graphs[(size_t)id];
  const unsigned blocks = blocks_for(g.n, 256, 4096);
  const int32_t base = (int32_t)g.base, n = (int32_t)g.n;
  if (p->tune.hook == 1) {
    hipLaunchKernelGGL(k_iota_i32, dim3(blocks), dim3(256), 0, p->stream, out, n);
    hipLaunchKernelGGL(k_pool_labels_min<false>, dim3(blocks), dim3(256), 0, p->stream, p->arena, base, n, out,
                       p->flags);
    hipLaunchKernelGGL(k_pool_labels_gather<false>, dim3(blocks), dim3(256), 0, p->stream, p->arena, base, n, out,
                       p->flags);
  } else if (p->tune.hook == 2) {
    hipLaunchKernelGGL(k_iota_i32, dim3(blocks), dim3(256), 0, p->stream, out, n);
    hipLaunchKernelGGL(k_pool_labels_min<true>, dim3(blocks), dim3(256), 0, p->stream, p->arena, base, n, out,
                       p->flags);
    hipLaunchKernelGGL(k_pool_labels_gather<true>, dim3(blocks), dim3(256), 0, p->stream, p->arena, base, n, out,
                       p->flags);
  } else {
    hipLaunchKernelGGL(k_pool_labels_id, dim3(blocks), dim3(256), 0, p->stream, p->arena, base, n, out, p->flags);
  }
  HIP_TRY(hipGetLastError());
  return CC_OK;
}

namespace {
int ensure_staging(cc_pool* p, int64_t n) {
  if (!p->check && hipMalloc(&p->check, 16) != hipSuccess) {
    p->check = nullptr;
    cc_set_error("image check buffer allocation failed");
    return CC_ENOMEM;
  }
  if (p->staging_cap >= n) return CC_OK;
  HIP_TRY(hipStreamSynchronize(p->stream));
  (void)hipFree(p->staging);
  p->staging = nullptr;
  p->staging_cap = 0;
  if (hipMalloc(&p->staging, (size_t)n * 4) != hipSuccess) {
    p->staging = nullptr;
    cc_set_error("image staging allocation failed");
    return CC_ENOMEM;
  }
  p->staging_cap = n;
  return CC_OK;
}

int read_graph_links(cc_pool* p, int32_t id, unsigned long long* links) {
  HIP_TRY(hipMemcpyAsync(links, p->glinks + (size_t)id * kPoolLinkStride, 8, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return CC_OK;
}
}  // namespace

extern "C" int cc_pool_num_components(cc_pool* p, int32_t id, int64_t* out) {
  if (!valid_graph(p, id) || !out) return CC_EINVAL;
  DeviceGuard dg(p->device);
  unsigned long long links = 0;
  int rc = read_graph_links(p, id, &links);
  if (rc != CC_OK) return rc;
  *out = p->graphs[(size_t)id].n - (int64_t)links;
  return CC_OK;
}

extern "C" int cc_pool_sync(cc_pool* p) {
  if (!p) return CC_EINVAL;
  DeviceGuard dg(p->device);
  HIP_TRY(hipStreamSynchronize(p->stream));
  int f = 0;
  HIP_TRY(hipMemcpyAsync(&f, p->flags, sizeof(int), hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (f) {
    HIP_TRY(hipMemsetAsync(p->flags, 0, sizeof(int), p->stream));
    HIP_TRY(hipStreamSynchronize(p->stream));
  }
  if (f & kFlagCorrupt) {
    cc_set_error("a find exceeded n steps: a forest in the pool holds a cycle");
    return CC_ECORRUPT;
  }
  if (f & kFlagRange) {
    cc_set_error("an edge or pair held a vertex id outside its graph; it was skipped");
    return CC_ERANGE;
  }
  return CC_OK;
}

extern "C" int64_t cc_pool_state_bytes(const cc_pool* p, int32_t id) {
  return valid_graph(p, id) ? 16 + 4 * p->graphs[(size_t)id].n : 0;
}

extern "C" int cc_pool_save(cc_pool* p, int32_t id, void* host_buf) {
  if (!valid_graph(p, id) || !host_buf) return CC_EINVAL;
  DeviceGuard dg(p->device);
  const PoolGraph& g = p->graphs[(size_t)id];
  unsigned long long links = 0;
  int rc = read_graph_links(p, id, &links);
  if (rc != CC_OK) return rc;
  int64_t hdr[2] = {g.n, (int64_t)links};
  memcpy(host_buf, hdr, 16);
  // the graph's slots hold graph-local ids: they are the image as they are
  HIP_TRY(hipMemcpyAsync((char*)host_buf + 16, p->arena + g.base, (size_t)g.n * 4, hipMemcpyDeviceToHost,
                         p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  return CC_OK;
}

extern "C" int cc_pool_load(cc_pool* p, int32_t id, const void* host_buf) {
  if (!valid_graph(p, id) || !host_buf) return CC_EINVAL;
  DeviceGuard dg(p->device);
  const PoolGraph& g = p->graphs[(size_t)id];
  int64_t hdr[2];
  memcpy(hdr, host_buf, 16);
  if (hdr[0] != g.n) {
    cc_set_error("cc_pool_load: image has n=%lld, graph has n=%lld", (long long)hdr[0], (long long)g.n);
    return CC_EINVAL;
  }
  int rc = ensure_staging(p, p->tune.hook == 2 ? 2 * g.n : g.n);
  if (rc != CC_OK) return rc;
  const unsigned blocks = blocks_for(g.n, 256, 4096);
  HIP_TRY(hipMemcpyAsync(p->staging, (const char*)host_buf + 16, (size_t)g.n * 4, hipMemcpyHostToDevice,
                         p->stream));
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, p->stream, p->check, 2);
  if (p->tune.hook == 2) {
    // a rank image keeps ranks, not an order, in its words: every vertex must
    // reach a root by pointer doubling (scratch: the second half of staging)
    int32_t* r = p->staging + g.n;
    hipLaunchKernelGGL(k_rank_image_init, dim3(blocks), dim3(256), 0, p->stream, p->staging, (int32_t)g.n, r,
                       p->check);
    for (int k = 0; k < 32; ++k)
      hipLaunchKernelGGL(k_rank_image_jump, dim3(blocks), dim3(256), 0, p->stream, r, (int32_t)g.n);
    hipLaunchKernelGGL(k_rank_image_verify, dim3(blocks), dim3(256), 0, p->stream, p->staging, r, (int32_t)g.n,
                       p->check);
  } else {
    if (p->tune.hook == 1)
      hipLaunchKernelGGL(k_check_image<true>, dim3(blocks), dim3(256), 0, p->stream, p->staging, (int32_t)g.n,
                         p->check);
    else
      hipLaunchKernelGGL(k_check_image<false>, dim3(blocks), dim3(256), 0, p->stream, p->staging, (int32_t)g.n,
                         p->check);
  }
  HIP_TRY(hipGetLastError());
  unsigned long long res[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(res, p->check, 16, hipMemcpyDeviceToHost, p->stream));
  HIP_TRY(hipStreamSynchronize(p->stream));
  if (res[0] != 0 || hdr[1] != g.n - (int64_t)res[1]) {
    cc_set_error("cc_pool_load: image is not a forest under the pool's linking order");
    return CC_ECORRUPT;
  }
  unsigned long long links = (unsigned long long)hdr[1];
  HIP_TRY(hipMemcpyAsync(p->arena + g.base, p->staging, (size_t)g.n * 4, hipMemcpyDeviceToDevice, p->stream));
  HIP_TRY(hipMemcpyAsync(p->glinks + (size_t)id * kPoolLinkStride, &links, 8, hipMemcpyHostToDevice, p->stream));
  if (const int frc = filter_clear(p, g.base, g.n, id, id + 1)) return frc;
  p->unrefreshed[(size_t)id] = g.n;  // renew at the next update
  HIP_TRY(hipStreamSynchronize(p->stream));
  return CC_OK;
}

// C ABI of the plain path (include/cc.h): one graph, one launch set per bulk
// operation, all work stream ordered on the graph's HIP stream.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "../../include/cc.h"
#include "cc_internal.hpp"
#include "cc_kernels.hpp"
#include "cc_vertex_kernels.hpp"
#include "cc_bulkfind_kernels.hpp"
#include "cc_contract_kernels.hpp"
#include "cc_stream_kernels.hpp"
#include "cc_member_kernels.hpp"

using namespace ccdev;
using cc::blocks_for;
using cc::DeviceGuard;

namespace {
thread_local char g_err[512] = "";
}

void cc_set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

extern "C" const char* cc_last_error(void) { return g_err; }

namespace cc {
namespace {
struct CoopState {
  hipEvent_t last = nullptr;     // recorded after the last cooperative launch
  hipStream_t stream = nullptr;  // the stream it was issued on
  bool any = false;
};
constexpr int kMaxDevices = 64;
std::mutex g_coop_mu;
CoopState g_coop[kMaxDevices];
}  // namespace

int coop_before(hipStream_t stream) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return CC_OK;
  std::lock_guard<std::mutex> lk(g_coop_mu);
  CoopState& c = g_coop[dev];
  if (c.any && c.stream != stream) HIP_TRY(hipStreamWaitEvent(stream, c.last, 0));
  return CC_OK;
}

int coop_after(hipStream_t stream) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return CC_OK;
  std::lock_guard<std::mutex> lk(g_coop_mu);
  CoopState& c = g_coop[dev];
  if (!c.last) HIP_TRY(hipEventCreateWithFlags(&c.last, hipEventDisableTiming | hipEventDisableSystemFence));
  HIP_TRY(hipEventRecord(c.last, stream));
  c.stream = stream;
  c.any = true;
  return CC_OK;
}
}  // namespace cc

extern "C" const char* cc_strerror(int code) {
  switch (code) {
    case CC_OK: return "ok";
    case CC_EINVAL: return "invalid argument";
    case CC_ENOMEM: return "out of memory";
    case CC_ERANGE: return "vertex id out of range (item skipped)";
    case CC_EDEVICE: return "HIP device error";
    case CC_ECORRUPT: return "corrupt union-find forest";
    default: return "unknown status";
  }
}

// Scratch of cc_bulk_update_noalloc (layout and use at noalloc_scratch).
constexpr int64_t kNoAllocMaxEdges = int64_t(1) << 22;
constexpr int kNoAllocHeadWords = 64;
static __device__ __align__(256) int32_t scratch[kNoAllocHeadWords + kNoAllocMaxEdges];

struct cc_graph {
  int64_t n = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t* parent = nullptr;
  unsigned long long* slots = nullptr;  // kSlots spread link counters
  unsigned long long* red = nullptr;    // reduction result (count_roots)
  int* flags = nullptr;
  int2* live = nullptr;
  unsigned* live_ctl = nullptr;  // [0] live count, [1] finished blocks, [2..3] same for hooked
  unsigned* gbar = nullptr;      // device-wide barrier of cc_bulk_stream (kBarWords)
  int32_t* hooked = nullptr;     // roots linked by the last fused update (n entries)
  unsigned* contract_ctl = nullptr;  // survivor counters + barrier of the contracting update
  BulkFindScratch bf{};          // Bulk-Find scratch (allocated on first use)
  bool bf_ready = false;
  int64_t bf_seg0_entries = 0;   // allocated level-0 entries
  uint32_t* member = nullptr;    // membership bitmap of the filter, ceil(n / 32) words
  int32_t* member_ctl = nullptr; // kMemberCtlWords: anchor, refill request, touched-complete flag
  int64_t member_calls = 0;      // fused updates since the filter state was last reset
  int64_t bf_unrenewed = 0;      // Bulk-Find with the filter: update edges since the bits were last refilled
  bool pristine = true;          // no update or load since creation or the last reset
  bool touched_maybe_complete = false;  // the device's touched-complete flag may be set
  int64_t live_cap = 0;
  int64_t updates = 0;
  bool capturing = false;
  // compaction threshold (CC_OPT_SPLIT_BELOW): link-counter snapshots copied
  // to pinned host memory after updates, read once their copies finished
  struct Snap {
    unsigned long long* host = nullptr;  // kSlots * kSlotStride words, pinned
    hipEvent_t done = nullptr;
    bool pending = false;
    int64_t epoch = 0;    // reset count when taken
    int64_t edges = 0;    // edges of all updates since the reset, up to this one
  } snap[2];
  int snap_next = 0;
  int64_t epoch = 0;          // cc_reset / cc_load count
  int64_t epoch_edges = 0;    // edges since the last reset
  int64_t base_links = 0, base_edges = 0;  // the last snapshot read, in this epoch
  bool base_valid = true;     // base_links / base_edges describe the same moment
  double live_est = 1.0;      // estimated live fraction (links per edge) of recent updates
  bool split_now = false;     // the schedule chosen by the last eager decision
  // effect of the calls recorded so far in the current capture on the
  // forest: a reset was recorded; updates recorded since the last reset (or
  // since the capture began)
  bool cap_reset = false;
  int64_t cap_updates = 0;
  cc::Tuning tune;
};

struct cc_exec {
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
  cc_graph* graph = nullptr;  // the graph it was captured on
  int hook = 0;               // linking order the recorded kernels were built for
  bool resets = false;        // the recording holds a reset ...
  int64_t updates = 0;        // ... and this many updates after its last reset (or in all)
  const uint32_t* member = nullptr;  // the filter bitmaps the recorded kernels keep (null: none)
};

namespace {

int alloc_live(cc_graph* g, int64_t cap) {
  if (cap <= g->live_cap) return CC_OK;
  if (g->live) {
    HIP_TRY(hipStreamSynchronize(g->stream));
    HIP_TRY(hipFree(g->live));
    g->live = nullptr;
    g->live_cap = 0;
  }
  if (hipMalloc(&g->live, (size_t)cap * sizeof(int2)) != hipSuccess) {
    g->live = nullptr;
    cc_set_error("hipMalloc of %lld live pairs failed", (long long)cap);
    return CC_ENOMEM;
  }
  g->live_cap = cap;
  return CC_OK;
}

int alloc_hooked(cc_graph* g) {
  if (g->hooked) return CC_OK;
  if (hipMalloc(&g->hooked, (size_t)g->n * sizeof(int32_t)) != hipSuccess) {
    g->hooked = nullptr;
    cc_set_error("hipMalloc of %lld hooked entries failed", (long long)g->n);
    return CC_ENOMEM;
  }
  return CC_OK;
}

void free_rd(cc_graph* g) {
  BulkFindScratch& b = g->bf;
  (void)hipFree(b.rd_cnt);
  (void)hipFree(b.rd_off);
  (void)hipFree(b.rd_pairs);
  (void)hipFree(b.rd_down);
  (void)hipFree(b.rd_big);
  b.rd_cnt = b.rd_off = nullptr;
  b.rd_pairs = b.rd_down = nullptr;
  b.rd_big = nullptr;
  b.rd_cap = 0;
}

// The response distributor's arrays for trails of up to cap entries (about
// 52 bytes per entry, plus 4 MiB of root-chunk padding).
int alloc_rd(cc_graph* g, int64_t cap) {
  BulkFindScratch& b = g->bf;
  if (b.rd_cap >= cap) return CC_OK;
  if (cap > 0x7fffffffLL) {
    cc_set_error("Bulk-Find with the response distributor: a trail bound of %lld entries exceeds 2^31 - 1",
                 (long long)cap);
    return CC_EINVAL;
  }
  HIP_TRY(hipStreamSynchronize(g->stream));
  free_rd(g);
  const size_t words = 3 * (size_t)cap + 1;
  bool ok = hipMalloc(&b.rd_cnt, words * 4) == hipSuccess && hipMalloc(&b.rd_off, words * 4) == hipSuccess &&
            hipMalloc(&b.rd_pairs, (size_t)cap * sizeof(int2)) == hipSuccess &&
            hipMalloc(&b.rd_down, (2 * (size_t)cap + (size_t)kRdRootPad) * sizeof(int2)) == hipSuccess &&
            hipMalloc(&b.rd_big, (size_t)cap * 4) == hipSuccess;
  if (!ok) {
    free_rd(g);
    cc_set_error("Bulk-Find: response distributor allocation (%lld entries) failed", (long long)cap);
    return CC_ENOMEM;
  }
  b.rd_cap = cap;
  return CC_OK;
}

void free_bulkfind(cc_graph* g) {
  BulkFindScratch& b = g->bf;
  free_rd(g);
  (void)hipFree(b.visited);
  (void)hipFree(b.seg0);
  (void)hipFree(b.log);
  (void)hipFree(b.ctl);
  (void)hipFree(b.open);
  (void)hipFree(b.seg_n);
  b = BulkFindScratch{};
  g->bf_ready = false;
  g->bf_seg0_entries = 0;
}

// Bulk-Find keeps its visited bitmap all clear between calls; this
// (re)establishes that state.
void clear_bulkfind(cc_graph* g) {
  const size_t words = ((size_t)g->n + 31) / 32;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for((int64_t)words, 256, 4096)), dim3(256), 0, g->stream,
                     (int32_t*)g->bf.visited, (int32_t)words, 0);
}

int alloc_bulkfind(cc_graph* g) {
  if (g->bf_ready) return CC_OK;
  BulkFindScratch& b = g->bf;
  const size_t n = (size_t)g->n, words = (n + 31) / 32;
  b.log_cap = 2 * (int64_t)n + 1024;
  bool ok = hipMalloc(&b.visited, words * 4) == hipSuccess &&
            hipMalloc(&b.log, (size_t)b.log_cap * 4) == hipSuccess &&
            hipMalloc(&b.ctl, kBulkFindCtlWords * sizeof(unsigned)) == hipSuccess &&
            hipMalloc(&b.seg_n, 2 * (size_t)kBfLevel0MaxBlocks * sizeof(uint32_t)) == hipSuccess;
  if (!ok) {
    free_bulkfind(g);
    cc_set_error("Bulk-Find scratch allocation (about 8 bytes per vertex) failed");
    return CC_ENOMEM;
  }
  clear_bulkfind(g);
  HIP_TRY(hipGetLastError());
  g->bf_ready = true;
  return CC_OK;
}

int64_t member_words(const cc_graph* g) { return (g->n + 31) / 32; }

// No anchor and both bitmaps empty (kernels only, so it can be captured).
// touched_complete: 1 for the initial forest (every vertex alone), 0 for a
// loaded one.
void member_reset(cc_graph* g, int touched_complete) {
  const int64_t words = member_words(g);
  hipLaunchKernelGGL(k_member_ctl_reset, dim3(1), dim3(64), 0, g->stream, g->member_ctl, touched_complete);
  g->touched_maybe_complete = touched_complete != 0;
  hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(2 * words, 256, 4096)), dim3(256), 0, g->stream,
                     (int32_t*)g->member, (int32_t)(2 * words), 0);
  g->member_calls = 0;
  g->bf_unrenewed = 0;
}

// An update that does not keep the touched bitmap complete is about to run.
// Skipped when the flag is known to be clear already; a capture always
// records it, since a replay may follow a reset.
void member_touched_invalid(cc_graph* g) {
  if (!g->member || !(g->touched_maybe_complete || g->capturing)) return;
  hipLaunchKernelGGL(k_member_touched_invalid, dim3(1), dim3(64), 0, g->stream, g->member_ctl);
  g->touched_maybe_complete = false;
}

int alloc_member(cc_graph* g) {
  if (g->member) return CC_OK;
  // membership bitmap, then touched bitmap
  if (hipMalloc(&g->member, (size_t)member_words(g) * 8) != hipSuccess ||
      hipMalloc(&g->member_ctl, kMemberCtlWords * sizeof(int32_t)) != hipSuccess) {
    (void)hipFree(g->member);
    g->member = nullptr;
    g->member_ctl = nullptr;
    cc_set_error("hipMalloc of the membership filter (n / 4 bytes) failed");
    return CC_ENOMEM;
  }
  member_reset(g, g->pristine ? 1 : 0);
  HIP_TRY(hipGetLastError());
  return CC_OK;
}

// Re-pick the anchor before update calls 0, 1, 2, 4, 8, ... and every 64th.
template <bool R>
void member_pick(cc_graph* g, const int2* e, int64_t m) {
  const int64_t c = g->member_calls++;
  if ((c & (c - 1)) != 0 && c % 64 != 0) return;
  hipLaunchKernelGGL(k_anchor_pick<R>, dim3(1), dim3(kPickThreads), 0, g->stream, g->parent, e, m,
                     (int32_t)g->n, g->member_ctl, g->flags);
  hipLaunchKernelGGL(k_member_reseed<R>, dim3(blocks_for(g->n, 256, 1024)), dim3(256), 0, g->stream, g->parent,
                     (int32_t)g->n, g->member_ctl, g->member, member_words(g), g->flags);
}

int launch_init(cc_graph* g) {
  const unsigned blocks = blocks_for((g->n + 3) / 4, 256, 2048);
  hipLaunchKernelGGL(k_init, dim3(blocks), dim3(256), 0, g->stream, g->parent, g->n);
  hipLaunchKernelGGL(k_zero_u64, dim3(4), dim3(256), 0, g->stream, g->slots, kSlots * kSlotStride);
  if (g->bf_ready) clear_bulkfind(g);
  if (g->member) member_reset(g, 1);
  g->pristine = true;
  HIP_TRY(hipGetLastError());
  return CC_OK;
}

// The fused update; with RECORD the roots it links go to `hooked`, counted in
// hooked_ctl[0] (hooked_ctl[1]: completion counter of the compress pass).
template <int ITEMS, class Ord, bool RECORD, bool FILT>
void launch_fused_t(cc_graph* g, const int2* e, int64_t m, int32_t* hooked, unsigned* hooked_ctl) {
  const int B = g->tune.block;
  const unsigned blocks = blocks_for(m, (int64_t)B * ITEMS, g->tune.grid_cap);
  hipLaunchKernelGGL((k_update_fused<ITEMS, Ord, RECORD, FILT>), dim3(blocks), dim3(B), 0, g->stream, g->parent,
                     e, m, (int32_t)g->n, g->slots, g->flags, hooked, hooked_ctl, g->member_ctl, g->member);
}

template <class Ord, bool RECORD, bool FILT>
void launch_fused_f(cc_graph* g, const int2* e, int64_t m, int32_t* hooked, unsigned* hooked_ctl) {
  int items = cc::pick_items(g->tune.items, m, g->tune.block);
  while (FILT && items > 1 && g->tune.block * items > kDeferTileMax) items >>= 1;  // a tile fits the list
  switch (items) {
    case 1: launch_fused_t<1, Ord, RECORD, FILT>(g, e, m, hooked, hooked_ctl); break;
    case 2: launch_fused_t<2, Ord, RECORD, FILT>(g, e, m, hooked, hooked_ctl); break;
    case 8: launch_fused_t<8, Ord, RECORD, FILT>(g, e, m, hooked, hooked_ctl); break;
    default: launch_fused_t<4, Ord, RECORD, FILT>(g, e, m, hooked, hooked_ctl); break;
  }
}

template <class Ord, bool RECORD>
void launch_fused_r(cc_graph* g, const int2* e, int64_t m, int32_t* hooked, unsigned* hooked_ctl) {
  if (g->tune.filter && g->member) {
    member_pick<is_ranked<Ord>::value>(g, e, m);
    launch_fused_f<Ord, RECORD, true>(g, e, m, hooked, hooked_ctl);
  } else {
    member_touched_invalid(g);
    launch_fused_f<Ord, RECORD, false>(g, e, m, hooked, hooked_ctl);
  }
}

// Fused update, then (with linked-root compression) the compress pass over
// the roots it linked.
template <class Ord>
void launch_fused_o(cc_graph* g, const int2* e, int64_t m) {
  if (g->tune.compress_linked) {
    launch_fused_r<Ord, true>(g, e, m, g->hooked, g->live_ctl + 2);
    const unsigned blocks = blocks_for(std::min<int64_t>(m, g->n), 256, 1024);
    hipLaunchKernelGGL(k_compress_hooked<is_ranked<Ord>::value>, dim3(blocks), dim3(256), 0, g->stream,
                       g->parent, g->hooked, g->live_ctl + 2, (int32_t)g->n, g->flags);
  } else {
    launch_fused_r<Ord, false>(g, e, m, nullptr, nullptr);
  }
}

template <int ITEMS, bool R>
void launch_filter_t(cc_graph* g, const int2* e, int64_t m) {
  const int B = g->tune.block;
  const unsigned blocks = blocks_for(m, (int64_t)B * ITEMS, g->tune.grid_cap);
  hipLaunchKernelGGL((k_filter<ITEMS, R>), dim3(blocks), dim3(B), (size_t)B * ITEMS * sizeof(int2), g->stream,
                     g->parent, e, m, (int32_t)g->n, g->live, g->live_ctl, g->flags);
}

template <class Ord>
void launch_split_o(cc_graph* g, const int2* e, int64_t m) {
  constexpr bool R = is_ranked<Ord>::value;
  switch (cc::pick_items(g->tune.items, m, g->tune.block)) {
    case 1: launch_filter_t<1, R>(g, e, m); break;
    case 2: launch_filter_t<2, R>(g, e, m); break;
    case 8: launch_filter_t<8, R>(g, e, m); break;
    default: launch_filter_t<4, R>(g, e, m); break;
  }
  const int B = g->tune.block;
  const unsigned blocks = blocks_for(m, B, g->tune.grid_cap);
  hipLaunchKernelGGL((k_link_live<Ord>), dim3(blocks), dim3(B), 0, g->stream, g->parent, g->live,
                     g->live_ctl, (int32_t)g->n, g->slots, g->flags);
  hipLaunchKernelGGL(k_compress_live<R>, dim3(blocks), dim3(B), 0, g->stream, g->parent, g->live, g->live_ctl,
                     (int32_t)g->n, g->flags);
}

template <int ITEMS, bool HALVE, bool R, bool FILT>
void launch_query_t(cc_graph* g, const int2* p, int64_t q, uint8_t* out) {
  const int B = g->tune.block;
  const unsigned blocks = blocks_for(q, (int64_t)B * ITEMS, g->tune.grid_cap);
  hipLaunchKernelGGL((k_query<ITEMS, HALVE, R, FILT>), dim3(blocks), dim3(B), 0, g->stream, g->parent, p, q,
                     (int32_t)g->n, out, g->flags, g->member_ctl, g->member);
}

template <bool HALVE, bool R, bool FILT>
void launch_query_f(cc_graph* g, const int2* p, int64_t q, uint8_t* out) {
  const int items = g->tune.query_items ? g->tune.query_items : g->tune.items;
  switch (cc::pick_items(items, q, g->tune.block)) {
    case 1: launch_query_t<1, HALVE, R, FILT>(g, p, q, out); break;
    case 2: launch_query_t<2, HALVE, R, FILT>(g, p, q, out); break;
    case 8: launch_query_t<8, HALVE, R, FILT>(g, p, q, out); break;
    default: launch_query_t<4, HALVE, R, FILT>(g, p, q, out); break;
  }
}

template <bool HALVE, bool R>
void launch_query_h(cc_graph* g, const int2* p, int64_t q, uint8_t* out) {
  if (g->tune.filter == 2 && g->member) launch_query_f<HALVE, R, true>(g, p, q, out);
  else launch_query_f<HALVE, R, false>(g, p, q, out);
}

unsigned vertex_blocks(const cc_graph* g) { return blocks_for(g->n, 256, 4096); }

int read_links(cc_graph* g, unsigned long long* links) {
  std::vector<unsigned long long> h((size_t)kSlots * kSlotStride);
  HIP_TRY(hipMemcpyAsync(h.data(), g->slots, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                         g->stream));
  HIP_TRY(hipStreamSynchronize(g->stream));
  unsigned long long s = 0;
  for (int i = 0; i < kSlots; ++i) s += h[(size_t)i * kSlotStride];
  *links = s;
  return CC_OK;
}

template <int KIND, class Ord, int PH2>
int launch_bulk_find_t(cc_graph* g, const int2* items, int64_t count, uint8_t* out, const uint32_t* member,
                       uint32_t* touched, const int32_t* member_ctl) {
  const int block = 256;
  int per_cu = 0, cus = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bulk_find<KIND, Ord, PH2>, block, 0));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
  // Phases I and II: one cooperative launch of at most kBfCoopBlocks blocks.
  // Its work is the trail, while each of its device-wide barriers costs
  // more the more blocks meet there (about 6 us at 256 blocks, 13 us at
  // 768): on the R-MAT stream 256 blocks beat 768 by 5-21% per pass, with
  // and without the membership filter, and beat 128.
  int64_t grid = (2 * count + block - 1) / block;
  grid = std::min<int64_t>(std::min<int64_t>(grid, cc::coop_limit(per_cu, cus, block)), kBfCoopBlocks);
  grid = std::max<int64_t>(1, std::min<int64_t>(grid, (int64_t)g->tune.grid_cap));
  // level 0: an ordinary launch of its own, about two items per thread, one
  // segment per block with room for both ends of its items
  const int64_t blocks0 =
      std::max<int64_t>(1, std::min<int64_t>((count + 2 * block - 1) / (2 * block), kBfLevel0MaxBlocks));
  const int64_t seg0_cap = 2 * ((count + blocks0 - 1) / blocks0);
  if (seg0_cap * blocks0 > g->bf_seg0_entries) {
    HIP_TRY(hipStreamSynchronize(g->stream));
    (void)hipFree(g->bf.seg0);
    (void)hipFree(g->bf.open);
    g->bf.seg0 = nullptr;
    g->bf.open = nullptr;
    g->bf_seg0_entries = 0;
    // the open-item lists take half as many entries as level 0
    if (hipMalloc(&g->bf.seg0, (size_t)(seg0_cap * blocks0) * 4) != hipSuccess ||
        hipMalloc(&g->bf.open, (size_t)(seg0_cap * blocks0 / 2) * 4) != hipSuccess) {
      (void)hipFree(g->bf.seg0);
      g->bf.seg0 = nullptr;
      g->bf.open = nullptr;
      cc_set_error("Bulk-Find: hipMalloc of %lld level-0 entries failed", (long long)(seg0_cap * blocks0));
      return CC_ENOMEM;
    }
    g->bf_seg0_entries = seg0_cap * blocks0;
  }
  g->bf.seg0_cap = seg0_cap;
  g->bf.seg_blocks = blocks0;
  if (PH2 == 1) {
    const int rc = alloc_rd(g, seg0_cap * blocks0 + g->bf.log_cap);
    if (rc != CC_OK) return rc;
  }
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, g->stream, g->bf.ctl, kBulkFindCtlWords);
  HIP_TRY(hipGetLastError());
  int32_t* parent = g->parent;
  int32_t n = (int32_t)g->n;
  BulkFindScratch sc = g->bf;
  // item indices of the open-item lists are 32-bit
  if (KIND != 0 || count > (int64_t)0xffffffffLL) sc.open = nullptr;
  unsigned long long* slots = g->slots;
  int* flags = g->flags;
  unsigned spin = (unsigned)g->tune.spin_limit;
  hipLaunchKernelGGL((k_bulk_find_level0<KIND>), dim3((unsigned)blocks0), dim3(block), 0, g->stream, items, count, n,
                     out, sc, flags, member, touched, member_ctl);
  HIP_TRY(hipGetLastError());
  void* args[] = {&parent, &items, &count, &n, &out, &sc, &slots, &flags, &spin, &member, &touched};
  if (const int crc = cc::coop_before(g->stream)) return crc;
  HIP_TRY(hipLaunchCooperativeKernel((const void*)k_bulk_find<KIND, Ord, PH2>, dim3((unsigned)grid), dim3(block),
                                     args, 0, g->stream));
  if (const int crc = cc::coop_after(g->stream)) return crc;
  return CC_OK;
}

int alloc_contract_ctl(cc_graph* g) {
  if (g->contract_ctl) return CC_OK;
  if (hipMalloc(&g->contract_ctl, (size_t)kContractCtlWords * sizeof(unsigned)) != hipSuccess) {
    g->contract_ctl = nullptr;
    cc_set_error("hipMalloc of the contracting update's counters failed");
    return CC_ENOMEM;
  }
  return CC_OK;
}

// Blocks of the contracting update's cooperative launch for m edges.
template <class Ord>
int contract_grid(cc_graph* g, int64_t m, int64_t* grid) {
  const int block = 256;
  int per_cu = 0, cus = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_contract<Ord>, block, 0));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
  // One block per 1024 edges up to 256 blocks, then one per 16K edges, at
  // most 1024: the rounds' device-wide barriers cost more the more blocks
  // meet at them, and only a huge minibatch has the work to pay for width
  // (R-MAT scale 24 in 64 / 8 / 1 minibatches, id order: 256, 512-1024 and
  // 1024 blocks were fastest, 14.3 / 11.3 / 25.3 ms per pass, against 24.9 /
  // 12.5 / 25.7 ms at the widest resident grid).
  int64_t b = (m + 4 * block - 1) / (4 * block);
  b = std::min<int64_t>(b, std::max<int64_t>(256, (m + 16383) / 16384));
  b = std::min<int64_t>(b, 1024);
  b = std::min<int64_t>(b, cc::coop_limit(per_cu, cus, block));
  b = std::min<int64_t>(b, (int64_t)g->tune.grid_cap);
  *grid = std::max<int64_t>(b, 1);
  return CC_OK;
}

template <class Ord>
int launch_contract_t(cc_graph* g, const int2* e, int64_t m) {
  int64_t grid = 0;
  int rc = contract_grid<Ord>(g, m, &grid);
  if (rc == CC_OK) rc = alloc_contract_ctl(g);
  int64_t seg_cap = (m + grid - 1) / grid;
  if (rc == CC_OK) rc = alloc_live(g, seg_cap * grid);
  if (rc != CC_OK) return rc;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, g->stream, g->contract_ctl, kContractCtlWords);
  HIP_TRY(hipGetLastError());
  int32_t* parent = g->parent;
  int32_t n = (int32_t)g->n;
  int2* list = g->live;
  unsigned* ctl = g->contract_ctl;
  unsigned long long* slots = g->slots;
  int* flags = g->flags;
  unsigned spin = (unsigned)g->tune.spin_limit;
  void* args[] = {&parent, &e, &m, &n, &list, &seg_cap, &ctl, &slots, &flags, &spin};
  if (const int crc = cc::coop_before(g->stream)) return crc;
  HIP_TRY(hipLaunchCooperativeKernel((const void*)k_contract<Ord>, dim3((unsigned)grid), dim3(256), args, 0,
                                     g->stream));
  if (const int crc = cc::coop_after(g->stream)) return crc;
  return CC_OK;
}

// Bulk-Find sets no membership bits, so before an update it refills them
// from `parent` (the anchor root and its direct children, which after a
// Bulk-Find are most of its trail) once n / 8 edges have gone in since the
// last refill, besides the anchor picks of the fused path's schedule.
template <bool R>
void bf_member_renew(cc_graph* g, const int2* e, int64_t m) {
  const int64_t c = g->member_calls++;
  const bool pick = (c & (c - 1)) == 0 || c % 64 == 0;
  const bool renew = 8 * g->bf_unrenewed >= g->n;
  if (pick)
    hipLaunchKernelGGL(k_anchor_pick<R>, dim3(1), dim3(kPickThreads), 0, g->stream, g->parent, e, m,
                       (int32_t)g->n, g->member_ctl, g->flags);
  if (renew) {
    hipLaunchKernelGGL(k_member_request_refill, dim3(1), dim3(64), 0, g->stream, g->member_ctl);
    g->bf_unrenewed = 0;
  }
  if (pick || renew)
    hipLaunchKernelGGL(k_member_reseed<R>, dim3(blocks_for(g->n, 256, 1024)), dim3(256), 0, g->stream, g->parent,
                       (int32_t)g->n, g->member_ctl, g->member, member_words(g), g->flags);
  g->bf_unrenewed += m;
}

// member: the membership bits Bulk-Find may settle items with, and the
// touched bitmap after them (updates with the filter on keep it; queries
// with filter 2 read it while the device flag says it is complete), or
// null.
template <int KIND>
int launch_bulk_find(cc_graph* g, const int2* items, int64_t count, uint8_t* out) {
  if (g->capturing) {
    cc_set_error("Bulk-Find is not available while capturing");
    return CC_EINVAL;
  }
  int rc = alloc_bulkfind(g);
  if (rc != CC_OK) return rc;
  const bool use = g->member && (KIND == 0 ? g->tune.filter != 0 : g->tune.filter == 2);
  const uint32_t* member = use ? g->member : nullptr;
  uint32_t* touched = use ? g->member + member_words(g) : nullptr;
  const int32_t* ctl = use ? g->member_ctl : nullptr;
  if (use && KIND == 0) {
    if (g->tune.hook == 2) bf_member_renew<true>(g, items, count);
    else bf_member_renew<false>(g, items, count);
    HIP_TRY(hipGetLastError());
  }
  if (g->tune.find == 2) {
    if (g->tune.hook == 1) return launch_bulk_find_t<KIND, ByHash, 1>(g, items, count, out, member, touched, ctl);
    if (g->tune.hook == 2) return launch_bulk_find_t<KIND, ByRank, 1>(g, items, count, out, member, touched, ctl);
    return launch_bulk_find_t<KIND, ById, 1>(g, items, count, out, member, touched, ctl);
  }
  if (g->tune.hook == 1) return launch_bulk_find_t<KIND, ByHash, 0>(g, items, count, out, member, touched, ctl);
  if (g->tune.hook == 2) return launch_bulk_find_t<KIND, ByRank, 0>(g, items, count, out, member, touched, ctl);
  return launch_bulk_find_t<KIND, ById, 0>(g, items, count, out, member, touched, ctl);
}

// Compaction threshold: fold finished link-counter snapshots into the
// live-fraction estimate and decide this update's schedule.
bool choose_split(cc_graph* g) {
  if (g->tune.split_below <= 0) return false;
  if (g->capturing) return g->split_now;
  for (int k = 0; k < 2; ++k) {
    cc_graph::Snap& sn = g->snap[(g->snap_next + k) % 2];  // older first
    if (!sn.pending || hipEventQuery(sn.done) != hipSuccess) continue;
    sn.pending = false;
    if (sn.epoch != g->epoch) continue;
    int64_t links = 0;
    for (int i = 0; i < kSlots; ++i) links += (int64_t)sn.host[(size_t)i * kSlotStride];
    if (g->base_valid && sn.edges > g->base_edges)
      g->live_est = (double)(links - g->base_links) / (double)(sn.edges - g->base_edges);
    g->base_links = links;
    g->base_edges = sn.edges;
    g->base_valid = true;
  }
  g->split_now = g->epoch_edges > 0 && g->live_est * 100.0 < (double)g->tune.split_below;
  return g->split_now;
}

// After an update under the threshold: copy the link counters to a free
// pinned slot (never waits; skipped when both slots are still in flight).
int snapshot_links(cc_graph* g, int64_t m) {
  g->epoch_edges += m;
  if (g->tune.split_below <= 0 || g->capturing) return CC_OK;
  cc_graph::Snap& sn = g->snap[g->snap_next];
  if (sn.pending) {
    if (hipEventQuery(sn.done) != hipSuccess) return CC_OK;
    (void)choose_split(g);  // fold it in before the slot is reused
  }
  if (!sn.host) {
    if (hipHostMalloc((void**)&sn.host, (size_t)kSlots * kSlotStride * 8, hipHostMallocDefault) != hipSuccess) {
      sn.host = nullptr;
      cc_set_error("pinned allocation of a link-counter snapshot failed");
      return CC_ENOMEM;
    }
    HIP_TRY(hipEventCreateWithFlags(&sn.done, hipEventDisableTiming));
  }
  HIP_TRY(hipMemcpyAsync(sn.host, g->slots, (size_t)kSlots * kSlotStride * 8, hipMemcpyDeviceToHost, g->stream));
  HIP_TRY(hipEventRecord(sn.done, g->stream));
  sn.pending = true;
  sn.epoch = g->epoch;
  sn.edges = g->epoch_edges;
  g->snap_next = (g->snap_next + 1) % 2;
  return CC_OK;
}

// A reset or load starts a new epoch of link counts (base: links 0, or the
// image's, at edge 0).  Updates whose edges the host does not count (the
// one-launch stream, Bulk-Find) also start one, with no base: the next
// snapshot read becomes the base.
void new_epoch(cc_graph* g, bool base_known = true) {
  g->epoch++;
  g->epoch_edges = 0;
  g->base_links = 0;
  g->base_edges = 0;
  g->base_valid = base_known;
  g->live_est = 1.0;
  g->split_now = false;
}

// Host state after an update call, and the periodic full compression.
void after_update(cc_graph* g) {
  g->updates++;
  g->pristine = false;
  if (g->capturing) g->cap_updates++;
  if (g->tune.compress_every > 0 && g->updates % g->tune.compress_every == 0) {
    if (g->tune.hook == 2)
      hipLaunchKernelGGL(k_compress_all<true>, dim3(vertex_blocks(g)), dim3(256), 0, g->stream, g->parent,
                         (int32_t)g->n, g->flags);
    else
      hipLaunchKernelGGL(k_compress_all<false>, dim3(vertex_blocks(g)), dim3(256), 0, g->stream, g->parent,
                         (int32_t)g->n, g->flags);
  }
}

// Scratch of cc_bulk_update_noalloc: words [0, 64) hold the count of the
// linked-root list and the completion counter of the compress pass (one
// 256-byte line), words [64, 64 + kNoAllocMaxEdges) hold the list (at most
// one linked root per edge).  Every device the library runs on holds its own
// copy until the process ends.  Host code never uses the array's name as an
// address: it asks the runtime for each device's address once
// (noalloc_scratch) and passes that.
constexpr int kNoAllocDevices = 64;
std::mutex g_scratch_mu;
int32_t* g_scratch_ptr[kNoAllocDevices] = {};

// Device address of `scratch` on the current device (looked up on the
// first call on each device).
int noalloc_scratch(int32_t** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kNoAllocDevices) {
    cc_set_error("cc_bulk_update_noalloc: device %d beyond the %d the library keeps scratch addresses for", dev,
                 kNoAllocDevices);
    return CC_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<int32_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return CC_OK;
}

template <class Ord>
void launch_fused_noalloc(cc_graph* g, const int2* e, int64_t m, int32_t* sc) {
  unsigned* ctl = reinterpret_cast<unsigned*>(sc);
  int32_t* list = sc + kNoAllocHeadWords;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, g->stream, ctl, 2);  // a kernel, not a memset node
  member_touched_invalid(g);
  launch_fused_f<Ord, true, false>(g, e, m, list, ctl);
  const unsigned blocks = blocks_for(std::min<int64_t>(m, g->n), 256, 1024);
  hipLaunchKernelGGL(k_compress_hooked<is_ranked<Ord>::value>, dim3(blocks), dim3(256), 0, g->stream, g->parent,
                     list, ctl, (int32_t)g->n, g->flags);
}

}  // namespace

// ---------------------------------------------------------------------------

extern "C" cc_graph* cc_create(int64_t n) {
  if (n < 1 || n > 0x7fffffffLL) {
    cc_set_error("cc_create: n=%lld outside [1, 2^31-1]", (long long)n);
    return nullptr;
  }
  cc_graph* g = new (std::nothrow) cc_graph();
  if (!g) {
    cc_set_error("cc_create: host allocation failed");
    return nullptr;
  }
  g->n = n;
  auto fail = [&](const char* what, hipError_t e) -> cc_graph* {
    cc_set_error("cc_create: %s: %s", what, hipGetErrorString(e));
    (void)hipFree(g->parent);
    (void)hipFree(g->slots);
    (void)hipFree(g->red);
    (void)hipFree(g->flags);
    (void)hipFree(g->live_ctl);
    (void)hipFree(g->gbar);
    delete g;
    return nullptr;
  };
  hipError_t e;
  if ((e = hipGetDevice(&g->device)) != hipSuccess) return fail("hipGetDevice", e);
  if ((e = hipMalloc(&g->parent, (size_t)n * sizeof(int32_t))) != hipSuccess) return fail("parent", e);
  if ((e = hipMalloc(&g->slots, (size_t)kSlots * kSlotStride * 8)) != hipSuccess) return fail("slots", e);
  if ((e = hipMalloc(&g->red, 64)) != hipSuccess) return fail("red", e);
  if ((e = hipMalloc(&g->flags, 64)) != hipSuccess) return fail("flags", e);
  if ((e = hipMalloc(&g->live_ctl, 64)) != hipSuccess) return fail("live_ctl", e);
  if ((e = hipMalloc(&g->gbar, kBarWords * sizeof(unsigned))) != hipSuccess) return fail("gbar", e);
  if ((e = hipMemsetAsync(g->flags, 0, 64, g->stream)) != hipSuccess) return fail("memset", e);
  if ((e = hipMemsetAsync(g->live_ctl, 0, 64, g->stream)) != hipSuccess) return fail("memset", e);
  if (launch_init(g) != CC_OK) return fail("init launch", hipGetLastError());
  if ((e = hipStreamSynchronize(g->stream)) != hipSuccess) return fail("sync", e);
  return g;
}

extern "C" int cc_destroy(cc_graph* g) {
  if (!g) return CC_EINVAL;
  if (g->capturing) {
    cc_set_error("call not allowed while capturing");
    return CC_EINVAL;
  }
  DeviceGuard dg(g->device);
  (void)hipStreamSynchronize(g->stream);
  (void)hipFree(g->parent);
  (void)hipFree(g->slots);
  (void)hipFree(g->red);
  (void)hipFree(g->flags);
  (void)hipFree(g->live);
  (void)hipFree(g->live_ctl);
  (void)hipFree(g->gbar);
  (void)hipFree(g->hooked);
  (void)hipFree(g->contract_ctl);
  (void)hipFree(g->member);
  (void)hipFree(g->member_ctl);
  if (g->bf_ready) free_bulkfind(g);
  for (auto& sn : g->snap) {
    if (sn.done) (void)hipEventDestroy(sn.done);
    if (sn.host) (void)hipHostFree(sn.host);
  }
  delete g;
  return CC_OK;
}

extern "C" int cc_set_stream(cc_graph* g, void* stream) {
  if (!g) return CC_EINVAL;
  g->stream = (hipStream_t)stream;
  return CC_OK;
}

extern "C" int cc_set_option(cc_graph* g, int key, int64_t value) {
  if (!g) return CC_EINVAL;
  if (key == CC_OPT_ONE_LAUNCH) {
    cc_set_error("cc_set_option: CC_OPT_ONE_LAUNCH applies to pools only");
    return CC_EINVAL;
  }
  if (key == CC_OPT_HOOK && value == 2 && g->n > (int64_t)kIdMask + 1) {
    cc_set_error("cc_set_option: union by rank needs n <= 2^%d", kRankShift);
    return CC_EINVAL;
  }
  // The forest's words and every label pass assume one linking order for
  // all links so far (rank bits sit in root words under union by rank).
  if (key == CC_OPT_HOOK && value != g->tune.hook && !g->pristine) {
    cc_set_error("cc_set_option: the linking order can change only before the first update after creation or "
                 "cc_reset");
    return CC_EINVAL;
  }
  if (!cc::set_tuning(&g->tune, key, value)) {
    cc_set_error("cc_set_option: key %d value %lld rejected", key, (long long)value);
    return CC_EINVAL;
  }
  return CC_OK;
}

extern "C" int cc_get_option(cc_graph* g, int key, int64_t* value) {
  if (!g || !value) return CC_EINVAL;
  if (!cc::get_tuning(&g->tune, key, value)) return CC_EINVAL;
  return CC_OK;
}

extern "C" int cc_reserve(cc_graph* g, int64_t max_batch) {
  if (!g || max_batch < 0) return CC_EINVAL;
  if (g->capturing) {
    cc_set_error("call not allowed while capturing");
    return CC_EINVAL;
  }
  DeviceGuard dg(g->device);
  int rc = alloc_hooked(g);
  if (rc == CC_OK && g->tune.filter) rc = alloc_member(g);
  if (rc != CC_OK) return rc;
  if (g->tune.mode == 2 && max_batch > 0) {
    int64_t grid = 0;
    rc = g->tune.hook == 1 ? contract_grid<ByHash>(g, max_batch, &grid) : contract_grid<ById>(g, max_batch, &grid);
    if (rc == CC_OK) rc = alloc_contract_ctl(g);
    if (rc != CC_OK) return rc;
    return alloc_live(g, (max_batch + grid - 1) / grid * grid);
  }
  return alloc_live(g, max_batch);
}

extern "C" int cc_reset(cc_graph* g) {
  if (!g) return CC_EINVAL;
  DeviceGuard dg(g->device);
  g->updates = 0;
  if (g->capturing) {
    g->cap_reset = true;
    g->cap_updates = 0;
  }
  new_epoch(g);
  return launch_init(g);
}

extern "C" int cc_bulk_update(cc_graph* g, const int32_t* edges, int64_t m) {
  if (!g || m < 0 || (m > 0 && (!edges || cc::misaligned8(edges)))) {
    cc_set_error("cc_bulk_update: invalid argument (edges must be 8-byte aligned device memory)");
    return CC_EINVAL;
  }
  if (m == 0) return CC_OK;
  DeviceGuard dg(g->device);
  const int2* e = reinterpret_cast<const int2*>(edges);
  if (g->tune.find != 0) {
    if (g->tune.filter && !g->member) {
      const int arc = alloc_member(g);
      if (arc != CC_OK) return arc;
    }
    if (!g->tune.filter) member_touched_invalid(g);  // with the filter, Bulk-Find keeps it
    int rc = launch_bulk_find<0>(g, e, m, nullptr);
    if (rc == CC_OK) {
      g->updates++;
      g->pristine = false;
      g->epoch_edges += m;
    }
    return rc;
  }
  const bool hashed = g->tune.hook == 1, ranked = g->tune.hook == 2;
  if (ranked && g->tune.mode == 2) {
    cc_set_error("cc_bulk_update: union by rank does not run with the contracting schedule");
    return CC_EINVAL;
  }
  if (g->tune.mode == 2) {
    if (g->capturing) {
      cc_set_error("cc_bulk_update: the contracting update is not available while capturing");
      return CC_EINVAL;
    }
    if (m > 0x7fffffffLL) {
      cc_set_error("cc_bulk_update: the contracting update takes at most 2^31-1 edges per call");
      return CC_EINVAL;
    }
    member_touched_invalid(g);
    int rc = hashed ? launch_contract_t<ByHash>(g, e, m) : launch_contract_t<ById>(g, e, m);
    if (rc != CC_OK) return rc;
  } else if (g->tune.mode == 1 ||
             (choose_split(g) && m <= 0x7fffffffLL && !(g->capturing && m > g->live_cap))) {
    if (m > 0x7fffffffLL) {  // the live count is a 32-bit device counter
      cc_set_error("cc_bulk_update: the split update takes at most 2^31-1 edges per call");
      return CC_EINVAL;
    }
    if (g->capturing && m > g->live_cap) {
      cc_set_error("cc_bulk_update: split update of %lld edges exceeds the reserved %lld during capture",
                   (long long)m, (long long)g->live_cap);
      return CC_EINVAL;
    }
    int rc = alloc_live(g, m);
    if (rc != CC_OK) return rc;
    member_touched_invalid(g);
    if (ranked) launch_split_o<ByRank>(g, e, m);
    else if (hashed) launch_split_o<ByHash>(g, e, m);
    else launch_split_o<ById>(g, e, m);
  } else {
    if (g->tune.compress_linked && !g->hooked) {
      if (g->capturing) {
        cc_set_error("cc_bulk_update: call cc_reserve before capturing");
        return CC_EINVAL;
      }
      int rc = alloc_hooked(g);
      if (rc != CC_OK) return rc;
    }
    if (g->tune.filter && !g->member) {
      if (g->capturing) {
        cc_set_error("cc_bulk_update: call cc_reserve before capturing");
        return CC_EINVAL;
      }
      int rc = alloc_member(g);  // still pristine if this is the graph's first update
      if (rc != CC_OK) return rc;
    }
    if (ranked) launch_fused_o<ByRank>(g, e, m);
    else if (hashed) launch_fused_o<ByHash>(g, e, m);
    else launch_fused_o<ById>(g, e, m);
  }
  after_update(g);
  HIP_TRY(hipGetLastError());
  return snapshot_links(g, m);
}

extern "C" int cc_bulk_update_noalloc(cc_graph* g, const int32_t* edges, int64_t m) {
  if (!g || m < 0 || (m > 0 && (!edges || cc::misaligned8(edges)))) {
    cc_set_error("cc_bulk_update_noalloc: invalid argument (edges must be 8-byte aligned device memory)");
    return CC_EINVAL;
  }
  if (m > kNoAllocMaxEdges) {
    cc_set_error("cc_bulk_update_noalloc: %lld edges exceed the limit of %lld per call", (long long)m,
                 (long long)kNoAllocMaxEdges);
    return CC_EINVAL;
  }
  if (m == 0) return CC_OK;
  DeviceGuard dg(g->device);
  int32_t* sc = nullptr;
  int rc = noalloc_scratch(&sc);
  if (rc != CC_OK) return rc;
  const int2* e = reinterpret_cast<const int2*>(edges);
  if (g->tune.hook == 2) launch_fused_noalloc<ByRank>(g, e, m, sc);
  else if (g->tune.hook == 1) launch_fused_noalloc<ByHash>(g, e, m, sc);
  else launch_fused_noalloc<ById>(g, e, m, sc);
  after_update(g);
  g->epoch_edges += m;
  HIP_TRY(hipGetLastError());
  return CC_OK;
}

extern "C" int cc_bulk_query(cc_graph* g, const int32_t* pairs, int64_t q, uint8_t* out) {
  if (!g || q < 0 || (q > 0 && (!pairs || !out || cc::misaligned8(pairs)))) {
    cc_set_error("cc_bulk_query: invalid argument (pairs must be 8-byte aligned device memory)");
    return CC_EINVAL;
  }
  if (q == 0) return CC_OK;
  DeviceGuard dg(g->device);
  const int2* p = reinterpret_cast<const int2*>(pairs);
  if (g->tune.find != 0) return launch_bulk_find<1>(g, p, q, out);
  const bool ranked = g->tune.hook == 2;
  if (g->tune.query_halving) {
    if (ranked) launch_query_h<true, true>(g, p, q, out);
    else launch_query_h<true, false>(g, p, q, out);
  } else {
    if (ranked) launch_query_h<false, true>(g, p, q, out);
    else launch_query_h<false, false>(g, p, q, out);
  }
  HIP_TRY(hipGetLastError());
  return CC_OK;
}

namespace {

template <bool FILT>
void launch_labels(cc_graph* g, int32_t* out) {
  const unsigned blocks = vertex_blocks(g);
  const int32_t n = (int32_t)g->n;
  const int32_t* mc = g->member_ctl;
  const uint32_t* mb = g->member;
  if (g->tune.hook == 0) {
    hipLaunchKernelGGL(k_labels_id<FILT>, dim3(blocks), dim3(256), 0, g->stream, g->parent, n, out, g->flags, mc, mb);
    return;
  }
  hipLaunchKernelGGL(k_iota_i32, dim3(blocks), dim3(256), 0, g->stream, out, n);
  if (g->tune.hook == 2) {
    hipLaunchKernelGGL((k_labels_min<true, FILT>), dim3(blocks), dim3(256), 0, g->stream, g->parent, n, out, g->flags,
                       mc, mb);
    hipLaunchKernelGGL((k_labels_gather<true, FILT>), dim3(blocks), dim3(256), 0, g->stream, g->parent, n, out,
                       g->flags, mc, mb);
  } else {
    hipLaunchKernelGGL((k_labels_min<false, FILT>), dim3(blocks), dim3(256), 0, g->stream, g->parent, n, out,
                       g->flags, mc, mb);
    hipLaunchKernelGGL((k_labels_gather<false, FILT>), dim3(blocks), dim3(256), 0, g->stream, g->parent, n, out,
                       g->flags, mc, mb);
  }
}

}  // namespace

// With the membership filter's bitmaps allocated, the label passes use them
// whatever the current options: they hold proofs either way.
extern "C" int cc_labels(cc_graph* g, int32_t* out) {
  if (!g || !out) return CC_EINVAL;
  DeviceGuard dg(g->device);
  if (g->member) launch_labels<true>(g, out);
  else launch_labels<false>(g, out);
  HIP_TRY(hipGetLastError());
  return CC_OK;
}

extern "C" int cc_num_components(cc_graph* g, int64_t* out) {
  if (!g || !out) return CC_EINVAL;
  if (g->capturing) {
    cc_set_error("call not allowed while capturing");
    return CC_EINVAL;
  }
  DeviceGuard dg(g->device);
  unsigned long long links = 0;
  int rc = read_links(g, &links);
  if (rc != CC_OK) return rc;
  *out = g->n - (int64_t)links;
  return CC_OK;
}

extern "C" int cc_count_roots(cc_graph* g, int64_t* out) {
  if (!g || !out) return CC_EINVAL;
  if (g->capturing) {
    cc_set_error("call not allowed while capturing");
    return CC_EINVAL;
  }
  DeviceGuard dg(g->device);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, g->stream, g->red, 1);
  if (g->tune.hook == 2)
    hipLaunchKernelGGL(k_count_roots<true>, dim3(vertex_blocks(g)), dim3(256), 0, g->stream, g->parent,
                       (int32_t)g->n, g->red);
  else
    hipLaunchKernelGGL(k_count_roots<false>, dim3(vertex_blocks(g)), dim3(256), 0, g->stream, g->parent,
                       (int32_t)g->n, g->red);
  HIP_TRY(hipGetLastError());
  unsigned long long h = 0;
  HIP_TRY(hipMemcpyAsync(&h, g->red, 8, hipMemcpyDeviceToHost, g->stream));
  HIP_TRY(hipStreamSynchronize(g->stream));
  *out = (int64_t)h;
  return CC_OK;
}

extern "C" int cc_filter_state(cc_graph* g, int32_t* anchor, int32_t* touched_complete, uint32_t* bits) {
  if (!g || !anchor || !touched_complete) return CC_EINVAL;
  if (g->capturing) {
    cc_set_error("call not allowed while capturing");
    return CC_EINVAL;
  }
  DeviceGuard dg(g->device);
  const size_t words = (size_t)member_words(g);
  if (!g->member) {
    *anchor = -1;
    *touched_complete = 0;
    if (bits) memset(bits, 0, 2 * words * 4);
    return CC_OK;
  }
  int32_t ctl[kMemberCtlWords];
  HIP_TRY(hipMemcpyAsync(ctl, g->member_ctl, sizeof(ctl), hipMemcpyDeviceToHost, g->stream));
  if (bits) HIP_TRY(hipMemcpyAsync(bits, g->member, 2 * words * 4, hipMemcpyDeviceToHost, g->stream));
  HIP_TRY(hipStreamSynchronize(g->stream));
  *anchor = ctl[0];
  *touched_complete = ctl[2];
  return CC_OK;
}

extern "C" int cc_sync(cc_graph* g) {
  if (!g) return CC_EINVAL;
  if (g->capturing) {
    cc_set_error("call not allowed while capturing");
    return CC_EINVAL;
  }
  DeviceGuard dg(g->device);
  HIP_TRY(hipStreamSynchronize(g->stream));
  int f = 0;
  HIP_TRY(hipMemcpyAsync(&f, g->flags, sizeof(int), hipMemcpyDeviceToHost, g->stream));
  HIP_TRY(hipStreamSynchronize(g->stream));
  if (f) {
    HIP_TRY(hipMemsetAsync(g->flags, 0, sizeof(int), g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
  }
  if (f & kFlagTimeout) {
    cc_set_error("a device-wide barrier of cc_bulk_stream timed out; its results are incomplete");
    return CC_EDEVICE;
  }
  if (f & kFlagCorrupt) {
    cc_set_error("a find exceeded n steps: the forest holds a cycle");
    return CC_ECORRUPT;
  }
  if (f & kFlagRange) {
    cc_set_error("an edge or pair held a vertex id outside [0, n); it was skipped");
    return CC_ERANGE;
  }
  return CC_OK;
}

extern "C" int64_t cc_num_vertices(const cc_graph* g) { return g ? g->n : 0; }

extern "C" int64_t cc_state_bytes(const cc_graph* g) { return g ? 16 + 4 * g->n : 0; }

extern "C" int cc_save(cc_graph* g, void* host_buf) {
  if (!g || !host_buf) return CC_EINVAL;
  if (g->capturing) {
    cc_set_error("call not allowed while capturing");
    return CC_EINVAL;
  }
  DeviceGuard dg(g->device);
  unsigned long long links = 0;
  int rc = read_links(g, &links);
  if (rc != CC_OK) return rc;
  int64_t hdr[2] = {g->n, (int64_t)links};
  memcpy(host_buf, hdr, 16);
  HIP_TRY(hipMemcpyAsync((char*)host_buf + 16, g->parent, (size_t)g->n * 4, hipMemcpyDeviceToHost, g->stream));
  HIP_TRY(hipStreamSynchronize(g->stream));
  return CC_OK;
}

extern "C" int cc_load(cc_graph* g, const void* host_buf) {
  if (!g || !host_buf) return CC_EINVAL;
  if (g->capturing) {
    cc_set_error("call not allowed while capturing");
    return CC_EINVAL;
  }
  DeviceGuard dg(g->device);
  int64_t hdr[2];
  memcpy(hdr, host_buf, 16);
  if (hdr[0] != g->n) {
    cc_set_error("cc_load: image has n=%lld, graph has n=%lld", (long long)hdr[0], (long long)g->n);
    return CC_EINVAL;
  }
  const int32_t* p = reinterpret_cast<const int32_t*>((const char*)host_buf + 16);
  int64_t roots = 0;
  if (!cc::check_forest(p, g->n, g->tune.hook, &roots) || hdr[1] != g->n - roots) {
    cc_set_error("cc_load: image is not a forest under the graph's linking order");
    return CC_ECORRUPT;
  }
  std::vector<unsigned long long> h((size_t)kSlots * kSlotStride, 0ull);
  h[0] = (unsigned long long)hdr[1];
  HIP_TRY(hipStreamSynchronize(g->stream));
  HIP_TRY(hipMemcpyAsync(g->parent, p, (size_t)g->n * 4, hipMemcpyHostToDevice, g->stream));
  HIP_TRY(hipMemcpyAsync(g->slots, h.data(), h.size() * 8, hipMemcpyHostToDevice, g->stream));
  if (g->member) member_reset(g, 0);  // its bits were proofs about the old forest
  g->pristine = false;
  new_epoch(g);
  g->base_links = hdr[1];
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(g->stream));
  return CC_OK;
}

extern "C" int cc_capture_begin(cc_graph* g) {
  if (!g || g->capturing || !g->stream) {
    cc_set_error("cc_capture_begin: needs a graph on a non-null stream, not already capturing");
    return CC_EINVAL;
  }
  DeviceGuard dg(g->device);
  int rc = alloc_hooked(g);  // allocations cannot happen inside the capture
  if (rc == CC_OK && g->tune.filter) rc = alloc_member(g);
  if (rc != CC_OK) return rc;
  HIP_TRY(hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal));
  g->capturing = true;
  g->cap_reset = false;
  g->cap_updates = 0;
  return CC_OK;
}

extern "C" int cc_capture_end(cc_graph* g, cc_exec** out) {
  if (!g || !out || !g->capturing) return CC_EINVAL;
  DeviceGuard dg(g->device);
  g->capturing = false;
  hipGraph_t graph = nullptr;
  HIP_TRY(hipStreamEndCapture(g->stream, &graph));
  cc_exec* x = new (std::nothrow) cc_exec();
  if (!x) {
    (void)hipGraphDestroy(graph);
    return CC_ENOMEM;
  }
  hipError_t e = hipGraphInstantiate(&x->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    cc_set_error("hipGraphInstantiate: %s", hipGetErrorString(e));
    delete x;
    return CC_EDEVICE;
  }
  x->stream = g->stream;
  x->device = g->device;
  x->graph = g;
  x->hook = g->tune.hook;
  x->resets = g->cap_reset;
  x->updates = g->cap_updates;
  x->member = g->member;
  *out = x;
  return CC_OK;
}

extern "C" int cc_exec_launch(cc_exec* x) {
  if (!x) return CC_EINVAL;
  cc_graph* g = x->graph;
  // The recorded kernels walk and link the forest under the linking order
  // of the capture; a forest built under another order (rank bits in root
  // words, other priorities) must not meet them.
  if (g->tune.hook != x->hook) {
    cc_set_error("cc_exec_launch: the graph's linking order changed since the capture");
    return CC_EINVAL;
  }
  if (g->capturing) {
    cc_set_error("cc_exec_launch: not allowed while the graph is capturing");
    return CC_EINVAL;
  }
  DeviceGuard dg(x->device);
  HIP_TRY(hipGraphLaunch(x->exec, x->stream));
  // The forest afterwards is what the recording leaves: no links only if it
  // resets and records no update after that, or if it neither resets nor
  // updates and the forest had none.
  if (x->resets) {
    g->pristine = x->updates == 0;
    g->updates = x->updates;
  } else if (x->updates > 0) {
    g->pristine = false;
    g->updates += x->updates;
  }
  if (x->resets || x->updates > 0) new_epoch(g, false);  // the replay's edge counts are not the host's
  // Filter bitmaps allocated after the capture were not kept by the
  // recorded kernels: after a recorded reset their bits are no proofs about
  // the new forest, and recorded updates may have linked vertices the
  // touched bitmap does not hold.
  if (g->member && g->member != x->member) {
    if (x->resets) member_reset(g, x->updates == 0 ? 1 : 0);
    else if (x->updates > 0) member_touched_invalid(g);
    HIP_TRY(hipGetLastError());
  }
  g->touched_maybe_complete = true;  // the replay may have reset the graph
  return CC_OK;
}

extern "C" int cc_exec_destroy(cc_exec* x) {
  if (!x) return CC_EINVAL;
  DeviceGuard dg(x->device);
  (void)hipStreamSynchronize(x->stream);
  (void)hipGraphExecDestroy(x->exec);
  delete x;
  return CC_OK;
}

namespace {

template <class Ord>
int launch_stream(cc_graph* g, int64_t batches, const int32_t* edges, const int64_t* eoff, const int32_t* pairs,
                  const int64_t* qoff, uint8_t* out, int64_t max_items) {
  const int block = g->tune.block;
  int per_cu = 0, cus = 0;
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_stream<Ord>, block, 0));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
  int64_t grid = (max_items + block - 1) / block;
  grid = std::min<int64_t>(grid, cc::coop_limit(per_cu, cus, block));
  grid = std::min<int64_t>(grid, std::min<int64_t>(1024, (int64_t)g->tune.grid_cap));
  grid = std::max<int64_t>(grid, 1);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, g->stream, g->gbar, kBarWords);
  HIP_TRY(hipGetLastError());
  int32_t* parent = g->parent;
  const int2* e = reinterpret_cast<const int2*>(edges);
  const int2* p = reinterpret_cast<const int2*>(pairs);
  int32_t n = (int32_t)g->n;
  unsigned long long* slots = g->slots;
  int* flags = g->flags;
  unsigned* bar = g->gbar;
  unsigned spin = (unsigned)g->tune.spin_limit;
  void* args[] = {&parent, &batches, &e, &eoff, &p, &qoff, &out, &n, &slots, &flags, &bar, &spin};
  if (const int crc = cc::coop_before(g->stream)) return crc;
  HIP_TRY(hipLaunchCooperativeKernel((const void*)k_stream<Ord>, dim3((unsigned)grid), dim3(block), args, 0,
                                     g->stream));
  if (const int crc = cc::coop_after(g->stream)) return crc;
  return CC_OK;
}

}  // namespace

extern "C" int cc_bulk_stream(cc_graph* g, int64_t batches, const int32_t* edges, const int64_t* eoff,
                              const int32_t* pairs, const int64_t* qoff, uint8_t* out, int64_t max_items) {
  if (!g || batches < 0 || max_items < 1 ||
      (batches > 0 && (!edges || !eoff || !pairs || !qoff || !out || cc::misaligned8(edges) ||
                       cc::misaligned8(pairs)))) {
    cc_set_error("cc_bulk_stream: invalid argument (edges and pairs must be 8-byte aligned device memory)");
    return CC_EINVAL;
  }
  if (g->capturing) {
    cc_set_error("cc_bulk_stream: not available while capturing");
    return CC_EINVAL;
  }
  if (batches == 0) return CC_OK;
  DeviceGuard dg(g->device);
  g->pristine = false;
  new_epoch(g, false);  // its edge counts stay on the device
  member_touched_invalid(g);
  if (g->tune.hook == 1) return launch_stream<ByHash>(g, batches, edges, eoff, pairs, qoff, out, max_items);
  if (g->tune.hook == 2) return launch_stream<ByRank>(g, batches, edges, eoff, pairs, qoff, out, max_items);
  return launch_stream<ById>(g, batches, edges, eoff, pairs, qoff, out, max_items);
}

// One launch for a whole sequence of minibatches: for every k, Bulk-Update of
// edges [eoff[k], eoff[k+1]) and then Bulk-Query of pairs [qoff[k], qoff[k+1]),
// separated by device-wide barriers, so the order of Section 1 (each bulk
// operation completes before the next begins) holds without a kernel
// boundary per operation.  Meant for streams of many small minibatches,
// whose cost in separate launches is mostly launch and drain latency.
//
// The grid is launched cooperatively; the barrier between operations is
// grid_sync (cc_grid.hpp).
#pragma once

#include "cc_grid.hpp"
#include "cc_kernels.hpp"

namespace ccdev {
namespace {

template <class Ord>
__global__ void k_stream(int32_t* __restrict__ parent, int64_t batches, const int2* __restrict__ edges,
                         const int64_t* __restrict__ eoff, const int2* __restrict__ pairs,
                         const int64_t* __restrict__ qoff, uint8_t* __restrict__ out, int32_t n,
                         unsigned long long* __restrict__ slots, int* __restrict__ flags, unsigned* bar,
                         unsigned spin_limit) {
  constexpr bool R = is_ranked<Ord>::value;
  const int64_t gsize = (int64_t)gridDim.x * blockDim.x;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned gen = 0;
  int links = 0;
  for (int64_t b = 0; b < batches; ++b) {
    const int64_t e1 = eoff[b + 1];
    for (int64_t i = eoff[b] + gtid; i < e1; i += gsize) {
      const int2 e = ld_stream_pair(edges, i);
      if (!in_range(e, n)) {
        raise_flag(flags, kFlagRange);
        continue;
      }
      if (e.x == e.y) continue;
      const int32_t pu = ldp<R>(parent + e.x), pv = ldp<R>(parent + e.y);
      if (pu == pv || pu == e.y || pv == e.x) continue;
      const int32_t ru = find_halve_from<R>(parent, e.x, pu, n, flags);
      const int32_t rv = find_halve_from<R>(parent, e.y, pv, n, flags);
      if (ru != rv) links += link(parent, ru, rv, n, flags, Ord{}) >= 0;
    }
    if (!grid_sync(bar, gen, flags, spin_limit)) break;
    const int64_t q1 = qoff[b + 1];
    for (int64_t i = qoff[b] + gtid; i < q1; i += gsize) {
      const int2 e = ld_stream_pair(pairs, i);
      uint8_t a = 0;
      if (!in_range(e, n)) {
        raise_flag(flags, kFlagRange);
      } else if (e.x == e.y) {
        a = 1;
      } else {
        a = find_halve<R>(parent, e.x, n, flags) == find_halve<R>(parent, e.y, n, flags);
      }
      out[i] = a;
    }
    if (!grid_sync(bar, gen, flags, spin_limit)) break;
  }
  count_links(slots, links);
}

}  // namespace
}  // namespace ccdev

// One launch for a whole sequence of minibatches: for every k, Bulk-Update of
// edges [eoff[k], eoff[k+1]) and then Bulk-Query of pairs [qoff[k], qoff[k+1]),
// with the order of Section 1 (each bulk operation completes before the next
// begins) kept by device-wide barriers instead of a kernel boundary per
// operation.  Meant for streams of many small minibatches, whose cost in
// separate launches is mostly launch and drain latency.
//
// The relabel step of Algorithm 2 (both roots of every edge) reads the
// forest and changes no connectivity; only the links do.  So the finds of
// minibatch k+1 run in the same phase as the queries of minibatch k, which
// read the same forest G_k, and the links of k+1 follow in a phase of their
// own:
//
//   phase X_k: answer the pairs of query k; find the roots of update k+1's
//              edges (path halving only shortens paths inside trees of G_k)
//   barrier B1 (no fences): every query of k has been answered
//   phase Y_k: link the root pairs found in X_k (a root linked meanwhile by
//              another thread fails its compare-and-swap and the link
//              continues from its new parent, as in every update)
//   barrier B2 (release/acquire): every link of k+1 is visible to the
//              queries of k+1
//
// Each thread walks its query pair and its edge (four finds) in lock step,
// one round of parent reads per level, so a phase waits for the deepest of
// its four paths rather than for their sum.  Per minibatch this is one
// fenced and one fence-free barrier, against two fenced ones when the finds
// and links of an update share one phase.
//
// B1 needs no fences: no value written in X_k is needed in Y_k (halving
// stores only shorten paths and target non-roots, compare-and-swaps target
// roots), and every query read of X_k has returned (its value is stored in
// `out` before the block arrives) before any link of Y_k is issued.
//
// The grid is launched cooperatively; the barriers are grid_sync
// (cc_grid.hpp).  Edges and pairs beyond one per thread in a minibatch are
// handled the plain way: such edges are found and linked in Y_k, such pairs
// are answered in X_k.
#pragma once

#include "cc_grid.hpp"
#include "cc_kernels.hpp"

namespace ccdev {
namespace {

// Roots of x[0..N) with path halving, all walks advanced together: every
// round issues one parent read per unfinished walk before using any.  Walks
// with act[j] false keep x[j].  Lanes with nothing to read read entry 0.
template <int N, bool R>
__device__ __forceinline__ void roots_lockstep(int32_t* parent, int32_t (&x)[N], bool (&act)[N], int32_t cap,
                                               int* flags) {
  int32_t p[N];
#pragma unroll
  for (int j = 0; j < N; ++j) p[j] = ldp<R>(parent + (act[j] ? x[j] : 0));
  uint32_t steps = 0;
  for (;;) {
    bool any = false;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      act[j] = act[j] && p[j] != x[j];
      any = any || act[j];
    }
    if (!any) return;
    int32_t g[N];
#pragma unroll
    for (int j = 0; j < N; ++j) g[j] = ldp<R>(parent + (act[j] ? p[j] : 0));
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if (!act[j]) continue;
      if (g[j] == p[j]) {  // p is the root
        x[j] = p[j];
        act[j] = false;
      } else {
        st(parent + x[j], g[j]);
        x[j] = g[j];
      }
    }
#pragma unroll
    for (int j = 0; j < N; ++j) p[j] = ldp<R>(parent + (act[j] ? x[j] : 0));
    if (++steps > (uint32_t)cap) {
      raise_flag(flags, kFlagCorrupt);
      return;
    }
  }
}

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
  // Offsets and this thread's first edge and pair of the coming phase X are
  // read one phase ahead (the inputs never change), so that X starts with
  // its parent reads.  k = -1: no queries yet, only update 0.
  int64_t e0 = batches > 0 ? eoff[0] : 0, e1 = batches > 0 ? eoff[1] : 0, q0 = 0, q1 = 0;
  int2 e = e0 + gtid < e1 ? ld_stream_pair(edges, e0 + gtid) : make_int2(0, 0);
  int2 q = make_int2(0, 0);
  for (int64_t k = -1; k < batches; ++k) {
    const bool upd = k + 1 < batches;
    const int64_t ie = e0 + gtid, iq = q0 + gtid;
    const bool he = ie < e1, hq = iq < q1;
    // phase X_k
    const bool ve = he && in_range(e, n), vq = hq && in_range(q, n);
    if ((he && !ve) || (hq && !vq)) raise_flag(flags, kFlagRange);
    int32_t x[4] = {ve ? e.x : 0, ve ? e.y : 0, vq ? q.x : 0, vq ? q.y : 0};
    bool act[4] = {ve && e.x != e.y, ve && e.x != e.y, vq && q.x != q.y, vq && q.x != q.y};
    roots_lockstep<4, R>(parent, x, act, n, flags);
    if (hq) out[iq] = vq && x[2] == x[3];
    for (int64_t i = iq + gsize; i < q1; i += gsize) {
      const int2 p = ld_stream_pair(pairs, i);
      uint8_t a = 0;
      if (!in_range(p, n)) raise_flag(flags, kFlagRange);
      else a = p.x == p.y || find_halve<R>(parent, p.x, n, flags) == find_halve<R>(parent, p.y, n, flags);
      out[i] = a;
    }
    // the next phase X: edges of update k+2, pairs of query k+1
    const int64_t ne0 = k + 2 < batches ? eoff[k + 2] : 0, ne1 = k + 2 < batches ? eoff[k + 3] : 0;
    const int64_t nq0 = upd ? qoff[k + 1] : 0, nq1 = upd ? qoff[k + 2] : 0;
    const int2 ne = ne0 + gtid < ne1 ? ld_stream_pair(edges, ne0 + gtid) : make_int2(0, 0);
    const int2 nq = nq0 + gtid < nq1 ? ld_stream_pair(pairs, nq0 + gtid) : make_int2(0, 0);
    if (upd && e1 > e0) {  // links follow (uniform over the grid); else no barrier is needed
      if (q1 > q0 && !grid_sync<false>(bar, gen, flags, spin_limit)) break;  // B1
      // phase Y_k
      if (ve && x[0] != x[1]) links += link(parent, x[0], x[1], n, flags, Ord{}) >= 0;
      for (int64_t i = ie + gsize; i < e1; i += gsize) {
        const int2 f = ld_stream_pair(edges, i);
        if (!in_range(f, n)) {
          raise_flag(flags, kFlagRange);
          continue;
        }
        if (f.x == f.y) continue;
        const int32_t pu = ldp<R>(parent + f.x), pv = ldp<R>(parent + f.y);
        if (pu == pv || pu == f.y || pv == f.x) continue;
        const int32_t ru = find_halve_from<R>(parent, f.x, pu, n, flags);
        const int32_t rv = find_halve_from<R>(parent, f.y, pv, n, flags);
        if (ru != rv) links += link(parent, ru, rv, n, flags, Ord{}) >= 0;
      }
      if (!grid_sync<true>(bar, gen, flags, spin_limit)) break;  // B2
    }
    e0 = ne0;
    e1 = ne1;
    q0 = nq0;
    q1 = nq1;
    e = ne;
    q = nq;
  }
  count_links(slots, links);
}

}  // namespace
}  // namespace ccdev

// One launch for a whole sequence of minibatches: for every k, Bulk-Update of
// edges [eoff[k], eoff[k+1]) and then Bulk-Query of pairs [qoff[k], qoff[k+1]),
// separated by device-wide barriers, so the order of Section 1 (each bulk
// operation completes before the next begins) holds without a kernel
// boundary per operation.  Meant for streams of many small minibatches,
// whose cost in separate launches is mostly launch and drain latency.
//
// The grid is launched cooperatively (all blocks resident).  A barrier: the
// block's threads meet at a workgroup barrier, then one thread per block
// makes the block's writes visible device-wide (agent-scope release fence:
// every wavefront of the block has passed the workgroup barrier, so one
// fence covers them, as in the usual grid-sync construction), counts the
// block in, and either publishes the next generation (last arrival) or
// waits for it; it then drops stale cached lines (agent-scope acquire
// fence) before the block's threads continue.  One fence pair per block
// instead of one per wavefront: each fence writes back or invalidates the
// whole L2 of the XCD, and thousands of them per barrier dominated its cost.
// The arrival counter, the generation and the abort word sit on separate
// 128-byte lines, so waiting blocks polling the generation do not contend
// with arrivals.  Waiting is bounded: past the spin limit a block raises the
// timeout flag and the abort word, and every block leaves the kernel at its
// next barrier.
#pragma once

#include "cc_kernels.hpp"

namespace ccdev {
namespace {

// Barrier state: bar[0] arrivals (monotone within a launch), bar[32]
// generation, bar[64] abort; all zero at launch.
constexpr int kBarWords = 96;

__device__ __forceinline__ unsigned bar_load(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool grid_sync(unsigned* bar, unsigned& gen, int* flags, unsigned spin_limit) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned target = gen + 1;
    int good = 1;
    const unsigned arrived = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == gridDim.x * target) {
      __hip_atomic_store(bar + 32, target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (bar_load(bar + 32) < target) {
        __builtin_amdgcn_s_sleep(2);
        if ((++spins & 31u) == 0u) {
          if (bar_load(bar + 64) != 0u) {
            good = 0;
            break;
          }
          if (spins > spin_limit) {
            __hip_atomic_store(bar + 64, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            raise_flag(flags, kFlagTimeout);
            good = 0;
            break;
          }
        }
      }
    }
    if (bar_load(bar + 64) != 0u) good = 0;
    ok = good;
    gen = target;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok != 0;
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
  for (int64_t b = 0; b < batches; ++b) {
    const int64_t e1 = eoff[b + 1];
    for (int64_t i = eoff[b] + gtid; i < e1; i += gsize) {
      const int2 e = edges[i];
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
      const int2 e = pairs[i];
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

__global__ void k_zero_u32(unsigned* p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0u;
}

}  // namespace
}  // namespace ccdev

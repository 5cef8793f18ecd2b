// Grid-wide cooperation for the kernels that run as one cooperative launch
// (every block resident at once): the device-wide barrier, block-wide scans,
// spread counters and list appends.
//
// Device-wide barrier: the block's threads meet at a workgroup barrier, then
// one thread per block makes the block's writes visible device-wide
// (agent-scope release fence: every wavefront of the block has passed the
// workgroup barrier, so one fence covers them, as in the usual grid-sync
// construction), counts the block in, and either publishes the next
// generation (last arrival) or waits for it; it then drops stale cached
// lines (agent-scope acquire fence) before the block's threads continue.
// One fence pair per block instead of one per wavefront: each fence writes
// back or invalidates the whole L2 of the XCD, and thousands of them per
// barrier dominated its cost.  The arrival counter, the generation and the
// abort word sit on separate 128-byte lines, so waiting blocks polling the
// generation do not contend with arrivals.  Arrivals on one address are
// served one at a time (about 12 ns each), so a grid of kBarSubMin blocks or
// more counts in on kBarSub sub-counters (block b on b mod kBarSub), and only
// the last arrival of each sub-group counts in on the top counter; it first
// passes its sub-group's releases on with an acquire-release fence.  Waiting is bounded: past the
// spin limit a block raises the timeout flag and the abort word, and every
// block leaves the kernel at its next barrier.
//
// Appends: a device-scope atomic on one address is served one at a time
// (about 12 ns each on MI355X), so a list that every wavefront appends to
// through one counter is limited to about 85 M appends/s.  Lists here are
// filled per block (own segment, or chunks reserved a thousand entries at a
// time) and their sizes summed over kCountSlots counters 128 B apart.
#pragma once

#include "uf_device.hpp"

namespace ccdev {
namespace {

// Barrier state: bar[0] arrivals (monotone within a launch), bar[32]
// generation, bar[64] abort, bar[96 + 32 s] arrivals of sub-group s; all zero
// at launch.
constexpr int kBarSub = 16;
constexpr int kBarSubMin = 256;
constexpr int kBarWords = 96 + 32 * kBarSub;

__device__ __forceinline__ unsigned bar_load(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// FENCE = false: the same meeting point without the release and acquire
// fences, for a phase boundary across which no data has to flow (the caller
// states why); it still orders in time every access a block made before
// arriving against every access made after the barrier releases.
template <bool FENCE = true>
__device__ __forceinline__ bool grid_sync(unsigned* bar, unsigned& gen, int* flags, unsigned spin_limit) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (FENCE) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned target = gen + 1;
    int good = 1;
    bool last;
    if (gridDim.x < (unsigned)kBarSubMin) {
      const unsigned arrived = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
      last = arrived == gridDim.x * target;
    } else {
      const unsigned s = blockIdx.x % kBarSub;
      const unsigned members = (gridDim.x - s + kBarSub - 1) / kBarSub;
      const unsigned a = __hip_atomic_fetch_add(bar + 96 + 32 * s, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
      last = false;
      if (a == members * target) {
        // the sub-group's last arrival: its acquire half synchronizes with
        // the members' release fences, its release half with the top-level
        // last arrival's acquire fence below
        if (FENCE) __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        const unsigned t = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u;
        last = t == (unsigned)kBarSub * target;
      }
    }
    if (last) {
      // The last arrival passes the others' releases on: its acquire fence
      // synchronizes with every block's release fence (a large grid's:
      // every sub-group leader's acquire-release fence), their increments
      // being in the release sequence it read, and its release store of the
      // generation with every waiter's acquire fence below.
      if (FENCE) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(bar + 32, target, FENCE ? __ATOMIC_RELEASE : __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
    if (FENCE) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  return ok != 0;
}

__device__ __forceinline__ unsigned ld_count(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_count(unsigned* p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan of per-thread counts over the block; returns this thread's
// offset and the block total.  Every thread of the block calls it.
__device__ __forceinline__ int block_scan(int cnt, int* total, int* wave_off) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int incl = cnt;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  if (lane == 63) wave_off[wid] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < nw; ++w) {
      const int c = wave_off[w];
      wave_off[w] = acc;
      acc += c;
    }
    wave_off[16] = acc;
  }
  __syncthreads();
  const int off = wave_off[wid] + incl - cnt;
  *total = wave_off[16];
  __syncthreads();  // wave_off is reused by the next call
  return off;
}

// Per-round totals (list sizes): one group of kCountSlots counters per
// round, a ring of three groups, each block adding to the counter of its
// index mod kCountSlots.  Group r is read by every block at the start of
// round r, added to during round r - 1, and cleared (by block 0) at the start
// of round r - 2, after everyone read it at the start of round r - 3.  Totals
// stay below 2^31.
constexpr int kCountSlots = 32;
constexpr int kCountStride = 32;  // 128 B apart
constexpr int kCountWords = 3 * kCountSlots * kCountStride;

__device__ __forceinline__ unsigned* count_group(unsigned* ctl, int round) {
  return ctl + (round % 3) * kCountSlots * kCountStride;
}

// Block 0 clears the group that round + 2 adds to.
__device__ __forceinline__ void clear_group_ahead(unsigned* ctl, int round) {
  if (blockIdx.x == 0 && threadIdx.x < kCountSlots) st_count(count_group(ctl, round + 2) + threadIdx.x * kCountStride, 0u);
}

__device__ __forceinline__ unsigned group_total(unsigned* grp, int* red) {
  if (threadIdx.x < 64) {
    int v = threadIdx.x < kCountSlots ? (int)ld_count(grp + threadIdx.x * kCountStride) : 0;
    v = wave_sum(v);
    if (threadIdx.x == 0) *red = v;
  }
  __syncthreads();
  const unsigned t = (unsigned)*red;
  __syncthreads();
  return t;
}

__global__ void k_zero_u32(unsigned* p, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) p[i] = 0u;
}

}  // namespace
}  // namespace ccdev

// Memory-system microbenchmarks (include/cc_bench.h): random gathers,
// streaming reads, copies and random compare-and-swaps.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cc_bench.h"

namespace {

// Chris Wellons' "lowbias32" integer hash.
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ uint32_t wave_xor(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v ^= __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ void sink_xor(uint32_t* sink, uint32_t acc) {
  acc = wave_xor(acc);
  if ((threadIdx.x & 63) == 0) atomicXor(sink, acc);
}

constexpr int kUnroll = 4;

__global__ void k_gather(const int32_t* __restrict__ t, uint32_t mask, int64_t count, uint32_t seed,
                         uint32_t* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * kUnroll;
  uint32_t acc = 0;
  for (int64_t i0 = ((int64_t)blockIdx.x * blockDim.x) * kUnroll + threadIdx.x; i0 < count; i0 += stride) {
    uint32_t v[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      const int64_t i = i0 + (int64_t)k * blockDim.x;
      const uint32_t j = hash32(seed ^ (uint32_t)i ^ (uint32_t)(i >> 32) * 0x9e3779b9u) & mask;
      v[k] = i < count ? (uint32_t)t[j] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) acc ^= v[k];
  }
  sink_xor(sink, acc);
}

__global__ void k_stream_read(const int4* __restrict__ p, int64_t n16, uint32_t* __restrict__ sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
    const int4 v = p[i];
    acc ^= (uint32_t)(v.x ^ v.y ^ v.z ^ v.w);
  }
  sink_xor(sink, acc);
}

__global__ void k_copy(int4* __restrict__ d, const int4* __restrict__ s, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) d[i] = s[i];
}

__global__ void k_cas(int32_t* __restrict__ t, uint32_t mask, int64_t count, uint32_t seed) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const uint32_t j = hash32(seed ^ (uint32_t)i ^ (uint32_t)(i >> 32) * 0x9e3779b9u) & mask;
    atomicCAS(t + j, (int32_t)j, (int32_t)(j ^ 1u));
  }
}

bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

unsigned grid_for(int64_t items, int per_block) {
  int64_t b = (items + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 8192) b = 8192;
  return (unsigned)b;
}

int launched() { return hipGetLastError() == hipSuccess ? 0 : -4; }

}  // namespace

extern "C" int ccb_gather(const int32_t* table, int64_t n_table, int64_t count, uint32_t seed, uint32_t* sink,
                          void* stream) {
  if (!table || !sink || count < 0 || !pow2(n_table) || n_table > (1ll << 31)) return -1;
  if (count == 0) return 0;
  hipLaunchKernelGGL(k_gather, dim3(grid_for(count, 256 * kUnroll)), dim3(256), 0, (hipStream_t)stream, table,
                     (uint32_t)(n_table - 1), count, seed, sink);
  return launched();
}

extern "C" int ccb_stream_read(const void* buf, int64_t bytes, uint32_t* sink, void* stream) {
  if (!buf || !sink || bytes < 0 || bytes % 16) return -1;
  if (bytes == 0) return 0;
  hipLaunchKernelGGL(k_stream_read, dim3(grid_for(bytes / 16, 256)), dim3(256), 0, (hipStream_t)stream,
                     (const int4*)buf, bytes / 16, sink);
  return launched();
}

extern "C" int ccb_copy(void* dst, const void* src, int64_t bytes, void* stream) {
  if (!dst || !src || bytes < 0 || bytes % 16) return -1;
  if (bytes == 0) return 0;
  hipLaunchKernelGGL(k_copy, dim3(grid_for(bytes / 16, 256)), dim3(256), 0, (hipStream_t)stream, (int4*)dst,
                     (const int4*)src, bytes / 16);
  return launched();
}

extern "C" int ccb_cas(int32_t* table, int64_t n_table, int64_t count, uint32_t seed, void* stream) {
  if (!table || count < 0 || !pow2(n_table) || n_table > (1ll << 31)) return -1;
  if (count == 0) return 0;
  hipLaunchKernelGGL(k_cas, dim3(grid_for(count, 256)), dim3(256), 0, (hipStream_t)stream, table,
                     (uint32_t)(n_table - 1), count, seed);
  return launched();
}

extern "C" int ccb_event_create(void** ev) {
  if (!ev) return -1;
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return -4;
  *ev = (void*)e;
  return 0;
}

extern "C" int ccb_event_record(void* ev, void* stream) {
  if (!ev) return -1;
  return hipEventRecord((hipEvent_t)ev, (hipStream_t)stream) == hipSuccess ? 0 : -4;
}

extern "C" int ccb_event_elapsed_ms(void* start, void* stop, float* ms) {
  if (!start || !stop || !ms) return -1;
  if (hipEventSynchronize((hipEvent_t)stop) != hipSuccess) return -4;
  return hipEventElapsedTime(ms, (hipEvent_t)start, (hipEvent_t)stop) == hipSuccess ? 0 : -4;
}

extern "C" int ccb_event_destroy(void* ev) {
  if (!ev) return -1;
  return hipEventDestroy((hipEvent_t)ev) == hipSuccess ? 0 : -4;
}

// Passes over all vertices: min-id labels, full compression, root count.
#pragma once

#include "uf_device.hpp"

namespace ccdev {
namespace {  // kernels get internal linkage in every translation unit

// Id order: every root is its tree's smallest id, so the label is the root.
// Each vertex is also pointed straight at its root.
__global__ void k_labels_id(int32_t* __restrict__ parent, int32_t n, int32_t* __restrict__ out,
                            int* __restrict__ flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int32_t r = find_halve(parent, v, n, flags);
    if (ld(parent + v) != r) st(parent + v, r);
    out[v] = r;
  }
}

__global__ void k_fill_i32(int32_t* __restrict__ out, int32_t n, int32_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    out[v] = value;
  }
}

__global__ void k_iota_i32(int32_t* __restrict__ out, int32_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    out[v] = v;
  }
}

// Hashed or rank order, pass 1: the minimum id of each tree collects in its
// root's slot.  out is pre-filled with out[v] = v, so a root's slot starts at
// the root's own id and a root (most of them are singletons) needs no atomic.
template <bool R = false>
__global__ void k_labels_min(int32_t* __restrict__ parent, int32_t n, int32_t* __restrict__ out,
                             int* __restrict__ flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int32_t r = find_halve<R>(parent, v, n, flags);
    if (r == v) continue;
    if (ld(parent + v) != r) st(parent + v, r);
    // a big component's root slot is hit by millions of vertices: read it
    // first and only try the atomic while it may still go down (blocks run
    // roughly in id order, so the minimum arrives early)
    if (ld(out + r) > v) atomicMin(out + r, v);
  }
}

// Hashed order, pass 2: every vertex copies its root's minimum.  A root
// rewrites its own slot with the same value; non-root slots are never read.
template <bool R = false>
__global__ void k_labels_gather(const int32_t* __restrict__ parent, int32_t n, int32_t* __restrict__ out,
                                int* __restrict__ flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int32_t r = find_read<R>(parent, v, n, flags);
    out[v] = out[r];
  }
}

template <bool R = false>
__global__ void k_compress_all(int32_t* __restrict__ parent, int32_t n, int* __restrict__ flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int32_t r = find_halve<R>(parent, v, n, flags);
    if (r != v && ld(parent + v) != r) st(parent + v, r);
  }
}

template <bool R = false>
__global__ void k_count_roots(const int32_t* __restrict__ parent, int32_t n,
                              unsigned long long* __restrict__ result) {
  __shared__ int part[16];
  int c = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    c += pid<R>(parent[v]) == v;
  }
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += part[w];
    if (s) atomicAdd(result, s);
  }
}

}  // namespace
}  // namespace ccdev

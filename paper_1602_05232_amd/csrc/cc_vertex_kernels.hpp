// Passes over all vertices: min-id labels, full compression, root count.
//
// With FILT the label passes first consult the membership filter's bitmaps
// (cc_member_kernels.hpp), which hold proofs: a member is in the anchor's
// component, whose root is found once per thread; while the touched bitmap
// is complete, a vertex in neither bitmap is alone and is its own label.
// Only the other vertices are walked (and pointed at their root).
#pragma once

#include "cc_member_kernels.hpp"
#include "uf_device.hpp"

namespace ccdev {
namespace {  // kernels get internal linkage in every translation unit

// What the filter's bitmaps settle about v: 1 = a member (in the component
// of root ra), 2 = alone, 0 = unknown.
__device__ __forceinline__ int label_class(const uint32_t* member, const uint32_t* touched, int32_t v, int32_t ra,
                                           bool lone) {
  const bool m = ra >= 0 && bit_test(bit_word(member, v), v);
  if (m) return 1;
  if (lone && !bit_test(bit_word(member, v), v) && !bit_test(bit_word(touched, v), v)) return 2;
  return 0;
}

// Id order: every root is its tree's smallest id, so the label is the root.
// Each walked vertex is also pointed straight at its root.
template <bool FILT>
__global__ void k_labels_id(int32_t* __restrict__ parent, int32_t n, int32_t* __restrict__ out,
                            int* __restrict__ flags, const int32_t* __restrict__ member_ctl,
                            const uint32_t* __restrict__ member) {
  const int32_t ra = FILT ? anchor_root<false>(parent, member_ctl, n, flags) : -1;
  const bool lone = FILT && touched_complete(member_ctl);
  const uint32_t* touched = FILT ? member + (((int64_t)n + 31) >> 5) : nullptr;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int c = FILT ? label_class(member, touched, v, ra, lone) : 0;
    if (c) {
      out[v] = c == 1 ? ra : v;
      continue;
    }
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
// With FILT, members are reduced over the block and the block's minimum goes
// to the anchor root's slot with one atomic; alone vertices have nothing to
// add.  Every thread of the block reaches the reduction.
template <bool R, bool FILT>
__global__ void k_labels_min(int32_t* __restrict__ parent, int32_t n, int32_t* __restrict__ out,
                             int* __restrict__ flags, const int32_t* __restrict__ member_ctl,
                             const uint32_t* __restrict__ member) {
  __shared__ int32_t part[16];
  const int32_t ra = FILT ? anchor_root<R>(parent, member_ctl, n, flags) : -1;
  const bool lone = FILT && touched_complete(member_ctl);
  const uint32_t* touched = FILT ? member + (((int64_t)n + 31) >> 5) : nullptr;
  int32_t mmin = 0x7fffffff;  // smallest member id this thread saw
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int c = FILT ? label_class(member, touched, v, ra, lone) : 0;
    if (c == 1) mmin = v < mmin ? v : mmin;
    if (c) continue;
    const int32_t r = find_halve<R>(parent, v, n, flags);
    if (r == v) continue;
    if (ld(parent + v) != r) st(parent + v, r);
    // a big component's root slot is hit by millions of vertices: read it
    // first and only try the atomic while it may still go down (blocks run
    // roughly in id order, so the minimum arrives early)
    if (ld(out + r) > v) atomicMin(out + r, v);
  }
  if (FILT && ra >= 0) {  // uniform: ra >= 0 exactly when the anchor is set
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int32_t o = __shfl_xor(mmin, off, 64);
      mmin = o < mmin ? o : mmin;
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = mmin;
    __syncthreads();
    if (threadIdx.x == 0) {
      int32_t b = 0x7fffffff;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) b = part[w] < b ? part[w] : b;
      if (b < ra && ld(out + ra) > b) atomicMin(out + ra, b);
    }
  }
}

// Hashed or rank order, pass 2: every vertex copies its root's minimum.  A
// root rewrites its own slot with the same value; non-root slots are never
// read.  With FILT, a member copies the anchor root's slot and an alone
// vertex keeps its own id.
template <bool R, bool FILT>
__global__ void k_labels_gather(const int32_t* __restrict__ parent, int32_t n, int32_t* __restrict__ out,
                                int* __restrict__ flags, const int32_t* __restrict__ member_ctl,
                                const uint32_t* __restrict__ member) {
  const int32_t ra = FILT ? anchor_root<R>(parent, member_ctl, n, flags) : -1;
  const bool lone = FILT && touched_complete(member_ctl);
  const uint32_t* touched = FILT ? member + (((int64_t)n + 31) >> 5) : nullptr;
  const int32_t la = ra >= 0 ? out[ra] : 0;  // the anchor component's label (pass 1 is complete)
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)i;
    const int c = FILT ? label_class(member, touched, v, ra, lone) : 0;
    if (c == 1) {
      out[v] = la;
      continue;
    }
    if (c == 2) continue;  // out[v] == v already
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

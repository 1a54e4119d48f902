// Device helpers shared by the sweep kernels: lane-group reductions and the
// guarded maxima a check sweep publishes.
#pragma once

#include "gabp_internal.h"

namespace gabp {

template <int G, typename T>
__device__ __forceinline__ T gsum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

template <int G, typename T>
__device__ __forceinline__ T gmax(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, G));
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide maxima of four values (every thread of the block must call, once
// per kernel); thread 0 ends with them.
__device__ __forceinline__ void block_max4(double &d, double &x, double &dp, double &pm) {
  __shared__ double sh[4][kBlock / 64];
  d = wave_max(d);
  x = wave_max(x);
  dp = wave_max(dp);
  pm = wave_max(pm);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = d; sh[1][w] = x; sh[2][w] = dp; sh[3][w] = pm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    d = sh[0][0]; x = sh[1][0]; dp = sh[2][0]; pm = sh[3][0];
    for (int k = 1; k < kBlock / 64; ++k) {
      d = fmax(d, sh[0][k]); x = fmax(x, sh[1][k]); dp = fmax(dp, sh[2][k]); pm = fmax(pm, sh[3][k]);
    }
  }
}

// thread 0 writes the block maxima to part[blockIdx.x]
__device__ __forceinline__ void block_publish(double d, double x, double dp, double pm,
                                              BlockPartial *part) {
  block_max4(d, x, dp, pm);
  if (threadIdx.x == 0) {
    BlockPartial b;
    b.dmax = d; b.xmax = x; b.dpmax = dp; b.pmax = pm;
    part[blockIdx.x] = b;
  }
}

// As block_publish, but for launches with more workgroups than partial slots
// and for checks split over several launches: thread 0 raises slot
// blockIdx.x % nslots to the maxima with integer atomics (non-negative
// doubles order like their bit patterns; NaN and -0 count as 0, as fmax would
// drop them).  The slots start at zero and the readout clears them.
__device__ __forceinline__ void atomic_max_nonneg(double *p, double v) {
  v = v > 0.0 ? v : 0.0;
  atomicMax((unsigned long long *)p, (unsigned long long)__double_as_longlong(v));
}

__device__ __forceinline__ void slot_publish(double d, double x, double dp, double pm,
                                             BlockPartial *part, int nslots) {
  block_max4(d, x, dp, pm);
  if (threadIdx.x == 0) {
    BlockPartial *q = part + (blockIdx.x % nslots);
    atomic_max_nonneg(&q->dmax, d);
    atomic_max_nonneg(&q->xmax, x);
    atomic_max_nonneg(&q->dpmax, dp);
    atomic_max_nonneg(&q->pmax, pm);
  }
}

// The block's maxima stored to one given entry; callable several times per
// kernel by every thread of the block.
__device__ __forceinline__ void entry_store(double d, double x, double dp, double pm,
                                            BlockPartial *q) {
  block_max4(d, x, dp, pm);
  if (threadIdx.x == 0) {
    BlockPartial b;
    b.dmax = d; b.xmax = x; b.dpmax = dp; b.pmax = pm;
    *q = b;
  }
  __syncthreads();  // block_max4's buffer is free again
}

// act[0] = number of segments with done == 0, act[1..] = their indices in
// increasing order.  Every thread of the (kBlock-thread) block must call;
// thread k % kBlock must be the one that last wrote seg[k].done, or a barrier
// must separate the writes from the call.
__device__ __forceinline__ void seg_compact(const SegCtl *seg, int nseg, int32_t *act) {
  __shared__ int wcount[kBlock / 64];
  __shared__ int base;
  const int lane = threadIdx.x & 63, w = threadIdx.x / 64;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int k0 = 0; k0 < nseg; k0 += kBlock) {
    const int k = k0 + threadIdx.x;
    const bool on = k < nseg && seg[k].done == 0;
    const unsigned long long m = __ballot(on);
    if (lane == 0) wcount[w] = __popcll(m);
    __syncthreads();
    int at = base + __popcll(m & ((1ull << lane) - 1ull));
    for (int v = 0; v < w; ++v) at += wcount[v];
    if (on) act[1 + at] = k;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int v = 0; v < kBlock / 64; ++v) base += wcount[v];
    __syncthreads();
  }
  if (threadIdx.x == 0) act[0] = base;
}

// Non-temporal (streaming) access: data read or written once per launch,
// kept from displacing what the launch reads more than once.
template <typename V>
__device__ __forceinline__ V nt_load(const V *p) {
  using E = decltype(p->x);
  constexpr int N = sizeof(V) / sizeof(E);
  typedef E vec __attribute__((ext_vector_type(N)));
  const vec v = __builtin_nontemporal_load((const vec *)p);
  V out;
  __builtin_memcpy(&out, &v, sizeof(V));
  return out;
}
template <typename V>
__device__ __forceinline__ void nt_store(V *p, const V &x) {
  using E = decltype(p->x);
  constexpr int N = sizeof(V) / sizeof(E);
  typedef E vec __attribute__((ext_vector_type(N)));
  vec v;
  __builtin_memcpy(&v, &x, sizeof(V));
  __builtin_nontemporal_store(v, (vec *)p);
}

}  // namespace gabp

// Device helpers shared by the cpmdp kernels.
#pragma once

#include <hip/hip_ext.h>

#include "cpmdp_internal.h"

namespace cpm {

// Kernel launch, with the kernel's start / stop times recorded in tm's
// events when tm is given.
template <typename F, typename... Args>
inline void klaunch(F kernel, dim3 grid, dim3 block, size_t shmem, hipStream_t st,
                    const LaunchTiming* tm, Args... args) {
  if (tm)
    hipExtLaunchKernelGGL(kernel, grid, block, static_cast<uint32_t>(shmem), st, tm->start,
                          tm->stop, 0u, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, shmem, st, args...);
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, FastDiv d) {
  return (__umulhi(n, d.magic) + n) >> d.shift;
}

// Blocks are dispatched to the 8 XCDs round-robin (block b -> XCD b % 8).
// Renumber them so that each XCD walks one contiguous range of the logical
// block space: neighbouring tiles then share that XCD's L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb / kXcds, rem = nb % kXcds;
  const int x = b % kXcds, j = b / kXcds;
  return x * q + (x < rem ? x : rem) + j;
}

// max that keeps NaN (so a non-finite residual is reported, not hidden).
__device__ __forceinline__ double nanmax(double a, double b) {
  return (a != a || a > b) ? a : b;
}

// max that keeps NaN, in the residual's own precision.
template <typename R>
__device__ __forceinline__ R nanmax_t(R a, R b) {
  return (a != a || a > b) ? a : b;
}

// Block-wide max of v, folded into slot[blockIdx.x & spread_mask] (FP64 bit
// pattern; non-negative doubles order like their bits, NaN sorts above +inf).
// Spreading the atomics of a sweep over kSpread words keeps thousands of
// blocks from serialising on one address; the reader takes the max.  FP32
// residuals are reduced in FP32 (exact for a max) and widened once.
template <typename R>
__device__ __forceinline__ void block_max_to_slot(R v, unsigned long long* slot,
                                                  unsigned spread_mask = kSpread - 1) {
  __shared__ R part[16];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = nanmax_t(v, __shfl_xor(v, off));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    R m = part[0];
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 1; i < nw; ++i) m = nanmax_t(m, part[i]);
    atomicMax(slot + (blockIdx.x & spread_mask),
              static_cast<unsigned long long>(__double_as_longlong(static_cast<double>(m))));
  }
}

// Block-wide max of v stored to *dst (as FP64) by a plain store (no atomic):
// sweeps that run in chunks give each block its own word and reduce the
// words of a chunk in one small kernel afterwards, which is cheaper than
// thousands of atomics per sweep that serialise on the slot words.  An FP32
// sweep reduces in FP32 (the max of FP32 values is exact, and half the
// shuffles of an FP64 reduction: about 0.5 us less per 32^4 sweep).
template <typename R>
__device__ __forceinline__ void block_max_store(R v, double* dst) {
  __shared__ R part[16];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = nanmax_t(v, __shfl_xor(v, off));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    R m = part[0];
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 1; i < nw; ++i) m = nanmax_t(m, part[i]);
    *dst = static_cast<double>(m);
  }
}

__device__ __forceinline__ void block_sum_to_counter(unsigned v, unsigned int* ctr) {
  __shared__ unsigned part[16];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned m = 0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) m += part[i];
    if (m) atomicAdd(ctr, m);
  }
}

__device__ __forceinline__ bool is_terminal(const uint32_t* bits, int s) {
  return (bits[s >> 5] >> (s & 31)) & 1u;
}

// Order-preserving map of doubles to unsigned 64-bit keys (so that an
// unsigned atomic max gives the max of signed values), and its inverse.
__device__ __forceinline__ unsigned long long dkey(double v) {
  const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dkey_value(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
  return __longlong_as_double(static_cast<long long>(b));
}

// Midrange (max V + min V) / 2 from the keys [max V, max -V].
__device__ __forceinline__ float midrange(const unsigned long long* keys) {
  return static_cast<float>(0.5 * (dkey_value(keys[0]) - dkey_value(keys[1])));
}

__device__ __forceinline__ double tie_tol(const unsigned long long* vmax_bits) {
  const double vm = __longlong_as_double(static_cast<long long>(*vmax_bits));
  return kTieRel * (vm > 1.0 ? vm : 1.0);
}

// Running tie rule over actions visited in increasing index order: the
// candidate changes only when a later action exceeds the running maximum by
// more than tol, so among near-equal maxima the lowest index is kept.
template <typename T>
__device__ __forceinline__ void tie_update(T q, int act, T tol, T& best, int& bi) {
  if (q > best + tol || best != best) {
    best = q;
    bi = act;
  } else if (q > best) {
    best = q;
  }
}

}  // namespace cpm

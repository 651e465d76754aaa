// Small streaming kernels: fills (used instead of hipMemsetAsync so that the
// same launches can be captured into HIP graphs), precision conversions, the
// FP64 refinement update V += e, a sup-norm reduction and a policy check.
#include "common.cuh"

namespace cpm {

namespace {

constexpr int kUtilBlock = 256;

int util_grid(int64_t n) {
  int64_t b = (n + kUtilBlock - 1) / kUtilBlock;
  if (b > kMaxBlocks) b = kMaxBlocks;
  return static_cast<int>(b < 1 ? 1 : b);
}

__global__ void fill_u64_kernel(unsigned long long* p, int n, unsigned long long v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_u32_kernel(unsigned int* p, int n, unsigned int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_f32_kernel(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void f64_to_f32_kernel(const double* s, float* d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = static_cast<float>(s[i]);
}
__global__ void f32_to_f64_kernel(const float* s, double* d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = static_cast<double>(s[i]);
}
__global__ void add_f32_to_f64_kernel(double* d, const float* e, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] += static_cast<double>(e[i]);
}
__global__ void copy_i32_kernel(const int32_t* s, int32_t* d, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}
__global__ void maxabs_f64_kernel(const double* v, int64_t n, unsigned long long* slot) {
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = nanmax(m, fabs(v[i]));
  block_max_to_slot(m, slot, 0u);
}
__global__ void reduce_parts_kernel(const double* parts, int nb, unsigned long long* slots) {
  const double* p = parts + static_cast<size_t>(blockIdx.x) * nb;
  double m = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) m = nanmax(m, p[i]);
  __shared__ double part[kUtilBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = nanmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = part[0];
    for (int i = 1; i < kUtilBlock / 64; ++i) r = nanmax(r, part[i]);
    slots[static_cast<size_t>(blockIdx.x) * kSpread] =
        static_cast<unsigned long long>(__double_as_longlong(r));
  }
}
__global__ void check_policy_kernel(const int32_t* pi, int64_t n, int32_t A, unsigned int* bad) {
  unsigned c = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    c += (pi[i] < 0 || pi[i] >= A) ? 1u : 0u;
  block_sum_to_counter(c, bad);
}

// keys[0] = ordered key of max V, keys[1] = ordered key of max(-V).
// keys[0] = max key of V, keys[1] = max key of -V.  16-byte loads where V is
// aligned; the block reduces in LDS and issues one atomic per key, so a
// launch makes at most 2 * kMinmaxBlocks atomics on the two words.
constexpr int kMinmaxBlocks = 512;
__global__ __launch_bounds__(kUtilBlock) void minmax_keys_f32_kernel(const float* V, int64_t n,
                                                                     unsigned long long* keys) {
  unsigned long long hi = 0, lo = 0;
  auto take = [&](float x) {
    const double v = static_cast<double>(x);
    hi = max(hi, dkey(v));
    lo = max(lo, dkey(-v));
  };
  const int64_t gid = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int64_t n4 = (reinterpret_cast<uintptr_t>(V) % 16 == 0) ? n / 4 : 0;
  const float4* V4 = reinterpret_cast<const float4*>(V);
  for (int64_t i = gid; i < n4; i += stride) {
    const float4 v = V4[i];
    take(v.x);
    take(v.y);
    take(v.z);
    take(v.w);
  }
  for (int64_t i = 4 * n4 + gid; i < n; i += stride) take(V[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    hi = max(hi, static_cast<unsigned long long>(__shfl_xor(static_cast<long long>(hi), off)));
    lo = max(lo, static_cast<unsigned long long>(__shfl_xor(static_cast<long long>(lo), off)));
  }
  __shared__ unsigned long long part[2][kUtilBlock / 64];
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    part[0][wid] = hi;
    part[1][wid] = lo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kUtilBlock / 64; ++w) {
      hi = max(hi, part[0][w]);
      lo = max(lo, part[1][w]);
    }
    atomicMax(keys, hi);
    atomicMax(keys + 1, lo);
  }
}

// keys[0] = max over non-terminal states of (BV - V), keys[1] = max of (V - BV).
__global__ void shift_bounds_kernel(const double* V, const double* BV, const uint32_t* tbits,
                                    int64_t n, unsigned long long* keys) {
  unsigned long long hi = 0, lo = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if ((tbits[i >> 5] >> (i & 31)) & 1u) continue;
    const double r = BV[i] - V[i];
    hi = max(hi, dkey(r));
    lo = max(lo, dkey(-r));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    hi = max(hi, static_cast<unsigned long long>(__shfl_xor(static_cast<long long>(hi), off)));
    lo = max(lo, static_cast<unsigned long long>(__shfl_xor(static_cast<long long>(lo), off)));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(keys, hi);
    atomicMax(keys + 1, lo);
  }
}

__global__ void apply_shift_kernel(double* V, const double* BV, const uint32_t* tbits, int64_t n,
                                   double shift) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    V[i] = BV[i] + (((tbits[i >> 5] >> (i & 31)) & 1u) ? 0.0 : shift);
}

}  // namespace

void launch_shift_bounds(const double* V, const double* BV, const uint32_t* tbits, int64_t n,
                         unsigned long long* keys, hipStream_t st) {
  hipLaunchKernelGGL(shift_bounds_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, V, BV, tbits, n, keys);
}
void launch_minmax_keys_f32(const float* V, int64_t n, unsigned long long* keys, hipStream_t st) {
  hipLaunchKernelGGL(minmax_keys_f32_kernel, dim3(std::min(util_grid((n + 3) / 4), kMinmaxBlocks)),
                     dim3(kUtilBlock), 0, st, V, n, keys);
}
void launch_apply_shift(double* V, const double* BV, const uint32_t* tbits, int64_t n, double shift,
                        hipStream_t st) {
  hipLaunchKernelGGL(apply_shift_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, V, BV, tbits, n, shift);
}

void launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st) {
  hipLaunchKernelGGL(fill_u64_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, p, n, v);
}
void launch_fill_u32(unsigned int* p, int n, unsigned int v, hipStream_t st) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, p, n, v);
}
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t st) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, p, n, v);
}
void launch_f64_to_f32(const double* s, float* d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, s, d, n);
}
void launch_f32_to_f64(const float* s, double* d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(f32_to_f64_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, s, d, n);
}
void launch_add_f32_to_f64(double* d, const float* e, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(add_f32_to_f64_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, d, e, n);
}
void launch_copy_i32(const int32_t* s, int32_t* d, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(copy_i32_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, s, d, n);
}
void launch_maxabs_f64(const double* v, int64_t n, unsigned long long* slot, hipStream_t st) {
  hipLaunchKernelGGL(maxabs_f64_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, v, n, slot);
}
void launch_reduce_parts(const double* parts, int nb, int k, unsigned long long* slots,
                         hipStream_t st) {
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(k), dim3(kUtilBlock), 0, st, parts, nb, slots);
}
void launch_check_policy(const int32_t* pi, int64_t n, int32_t A, unsigned int* bad, hipStream_t st) {
  hipLaunchKernelGGL(check_policy_kernel, dim3(util_grid(n)), dim3(kUtilBlock), 0, st, pi, n, A, bad);
}

}  // namespace cpm

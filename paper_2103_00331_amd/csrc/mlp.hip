// Learned warm start: a 130 -> 256 -> 256 -> 1 ReLU MLP that maps per-state
// features of a 3-D GridWorld (normalised coordinates, the 5x5x5 window of
// rewards around the state, gamma and slip) to y with (1 - gamma) V(s) =
// 0.2 + 0.05 y.  The prediction divided by (1 - gamma) is the initial V of value iteration;
// the solver itself, its FP64 certificate and plain VI from zero are
// unchanged.
//
// Kernels: feature gather, one tiled FP32 GEMM (64x64 block tile, 4x4 per
// thread, LDS-staged 16-deep K slices) with fused epilogues (bias, bias+ReLU,
// ReLU-mask multiply), MSE loss/gradient, Adam, parameter init.  Random
// numbers (minibatch indices, initial weights) come from SplitMix64 (Steele,
// Lea & Flood, OOPSLA 2014) with the Box-Muller transform for normals.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "common.cuh"
#include "cpmdp_internal.h"
#include "handle.h"

namespace cpm {

constexpr int kF = 130;        // features
constexpr int kXS = 132;       // row stride of the workspace's feature rows (16-byte aligned rows)
constexpr int kH = 256;        // hidden width
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + kF * kH;
constexpr int64_t kOffW2 = kOffB1 + kH;
constexpr int64_t kOffB2 = kOffW2 + kH * kH;
constexpr int64_t kOffW3 = kOffB2 + kH;
constexpr int64_t kOffB3 = kOffW3 + kH;
constexpr int64_t kParams = kOffB3 + 1;   // 99,585

// Feature normalisation constants (fixed, part of the model definition).
constexpr float kRScale = 10.0f;              // rewards ~ N(0, 0.1) -> unit scale
constexpr float kGammaMean = 0.945f, kGammaScale = 1.0f / 0.026f;
constexpr float kSlipMean = 0.175f, kSlipScale = 1.0f / 0.072f;
// Output: (1 - gamma) V = kOutMean + kOutScale * y.
constexpr double kOutMean = 0.2, kOutScale = 0.05;

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__device__ __forceinline__ float u01(uint64_t r) {   // (0, 1]
  return (static_cast<float>(r >> 40) + 1.0f) * (1.0f / 16777216.0f);
}

// ------------------------------------------------------------------ GEMM
enum { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_RELU = 2, EPI_MASK = 3 };

// C[M x N] = op(A) op(B) (+ epilogue).  op(A) is M x K: A[m*lda + k], or
// A[k*lda + m] when TA.  op(B) is K x N: B[k*ldb + n], or B[n*ldb + k] when TB.
// Split over K (gridDim.z > 1, EPI_NONE only): slice z sums k in
// [z kc, (z + 1) kc) and writes its partial product to C + z * M * ldc.
template <bool TA, bool TB, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K, const float* __restrict__ A,
                                                   int lda, const float* __restrict__ B, int ldb,
                                                   float* __restrict__ C, int ldc,
                                                   const float* __restrict__ bias,
                                                   const float* __restrict__ mask, int ldm, int kc) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
  C += static_cast<int64_t>(blockIdx.z) * M * ldc;
  float acc[4][4] = {};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    for (int i = threadIdx.x; i < 64 * 16; i += 256) {
      const int r = TA ? (i & 63) : (i >> 4);      // m within tile
      const int c = TA ? (i >> 6) : (i & 15);      // k within tile
      const int gm = m0 + r, gk = k0 + c;
      float v = 0.f;
      if (gm < M && gk < ke) v = TA ? A[static_cast<int64_t>(gk) * lda + gm] : A[static_cast<int64_t>(gm) * lda + gk];
      As[c][r] = v;
    }
    for (int i = threadIdx.x; i < 64 * 16; i += 256) {
      const int r = TB ? (i & 15) : (i >> 6);      // k within tile
      const int c = TB ? (i >> 4) : (i & 63);      // n within tile
      const int gk = k0 + r, gn = n0 + c;
      float v = 0.f;
      if (gk < ke && gn < N) v = TB ? B[static_cast<int64_t>(gn) * ldb + gk] : B[static_cast<int64_t>(gk) * ldb + gn];
      Bs[r][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gm = m0 + ty * 4 + i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gn = n0 + tx * 4 + j;
      if (gn >= N) continue;
      float v = acc[i][j];
      if (EPI == EPI_BIAS || EPI == EPI_BIAS_RELU) v += bias[gn];
      if (EPI == EPI_BIAS_RELU) v = fmaxf(v, 0.f);
      if (EPI == EPI_MASK) v = mask[static_cast<int64_t>(gm) * ldm + gn] > 0.f ? v : 0.f;
      C[static_cast<int64_t>(gm) * ldc + gn] = v;
    }
  }
}

// C[M x N] = op(A) op(B) (+ epilogue) on the FP32 matrix cores
// (v_mfma_f32_16x16x4f32); operands and epilogues as in gemm_kernel, split
// over K the same way.  Four waves in a 2 x 2 grid each compute WM x WN tiles
// of 16 x 16; the block's op(A) (BM x 16) and op(B) (16 x BN) slices go
// through LDS, k in steps of 16 (zero-padded past K, M and N), each read from
// global memory along its contiguous index.  The next slices are loaded into
// registers while the matrix cores work on the current ones; a slice inside
// the matrix is loaded without per-element guards, so that its loads issue
// together.  Lane l = 16 g + c of one 16x16x4 product supplies
// A[i = c][k = g] and B[k = g][n = c]; its result register r holds
// D[i = 4 g + r][n = c].
typedef float mlp_f4 __attribute__((ext_vector_type(4)));

// VA / VB: the operand's leading dimension is a multiple of 4 and its base
// 16-byte aligned, so a full tile's slice of it is read with 16-byte loads
// (four consecutive words along the operand's contiguous index) instead of
// one word per load.
template <bool TA, bool TB, int WM, int WN, int EPI, bool VA, bool VB>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(int M, int N, int K,
                                                        const float* __restrict__ A, int lda,
                                                        const float* __restrict__ B, int ldb,
                                                        float* __restrict__ C, int ldc,
                                                        const float* __restrict__ bias,
                                                        const float* __restrict__ mask, int ldm,
                                                        int kc) {
  constexpr int BM = 32 * WM, BN = 32 * WN, KT = 16;
  constexpr int LA = BM * KT / 256, LB = KT * BN / 256;   // slice words per thread
  __shared__ float As[KT][BM + 4];
  __shared__ float Bs[KT][BN + 4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int wm = wv >> 1, wn = wv & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kb = blockIdx.z * kc, ke = min(K, kb + kc);
  C += static_cast<int64_t>(blockIdx.z) * M * ldc;
  // slice word i -> (row or column within the tile, k within the slice),
  // consecutive i along the operand's contiguous index
  auto amap = [](int i, int& r, int& kk) {
    if (TA) { r = i % BM; kk = i / BM; } else { r = i / KT; kk = i % KT; }
  };
  auto bmap = [](int i, int& kk, int& cc) {
    if (TB) { kk = i % KT; cc = i / KT; } else { kk = i / BN; cc = i % BN; }
  };
  auto aidx = [&](int gm, int gk) {
    return TA ? static_cast<int64_t>(gk) * lda + gm : static_cast<int64_t>(gm) * lda + gk;
  };
  auto bidx = [&](int gk, int gn) {
    return TB ? static_cast<int64_t>(gn) * ldb + gk : static_cast<int64_t>(gk) * ldb + gn;
  };
  mlp_f4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = mlp_f4{0.f, 0.f, 0.f, 0.f};
  float ra[LA], rb[LB];
  bool va = false, vb = false;   // the slice in ra / rb was read in groups of 4
  auto fetch = [&](int k0) {
    const bool ka = k0 + KT <= ke;
    va = VA && ka && m0 + BM <= M;
    vb = VB && ka && n0 + BN <= N;
    if (va) {
      // group i of 4 words -> (row or column, k) of its first word, the 4
      // words consecutive along the contiguous index (m for TA, else k)
#pragma unroll
      for (int q = 0; q < LA / 4; ++q) {
        const int i = threadIdx.x + q * 256;
        int r, kk;
        if (TA) { r = (i % (BM / 4)) * 4; kk = i / (BM / 4); }
        else { r = i / (KT / 4); kk = (i % (KT / 4)) * 4; }
        const float4 v = *reinterpret_cast<const float4*>(A + aidx(m0 + r, k0 + kk));
        ra[4 * q] = v.x; ra[4 * q + 1] = v.y; ra[4 * q + 2] = v.z; ra[4 * q + 3] = v.w;
      }
    } else if (ka && m0 + BM <= M) {
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        int r, kk;
        amap(threadIdx.x + q * 256, r, kk);
        ra[q] = A[aidx(m0 + r, k0 + kk)];
      }
    } else {
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        int r, kk;
        amap(threadIdx.x + q * 256, r, kk);
        const int gm = m0 + r, gk = k0 + kk;
        ra[q] = (gm < M && gk < ke) ? A[aidx(gm, gk)] : 0.f;
      }
    }
    if (vb) {
#pragma unroll
      for (int q = 0; q < LB / 4; ++q) {
        const int i = threadIdx.x + q * 256;
        int kk, cc;
        if (TB) { kk = (i % (KT / 4)) * 4; cc = i / (KT / 4); }
        else { kk = i / (BN / 4); cc = (i % (BN / 4)) * 4; }
        const float4 v = *reinterpret_cast<const float4*>(B + bidx(k0 + kk, n0 + cc));
        rb[4 * q] = v.x; rb[4 * q + 1] = v.y; rb[4 * q + 2] = v.z; rb[4 * q + 3] = v.w;
      }
    } else if (ka && n0 + BN <= N) {
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        int kk, cc;
        bmap(threadIdx.x + q * 256, kk, cc);
        rb[q] = B[bidx(k0 + kk, n0 + cc)];
      }
    } else {
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        int kk, cc;
        bmap(threadIdx.x + q * 256, kk, cc);
        const int gk = k0 + kk, gn = n0 + cc;
        rb[q] = (gk < ke && gn < N) ? B[bidx(gk, gn)] : 0.f;
      }
    }
  };
  if (kb < ke) fetch(kb);
  for (int k0 = kb; k0 < ke; k0 += KT) {
    if (VA && va) {
#pragma unroll
      for (int q = 0; q < LA / 4; ++q) {
        const int i = threadIdx.x + q * 256;
        int r, kk;
        if (TA) { r = (i % (BM / 4)) * 4; kk = i / (BM / 4); }
        else { r = i / (KT / 4); kk = (i % (KT / 4)) * 4; }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (TA) As[kk][r + e] = ra[4 * q + e];
          else As[kk + e][r] = ra[4 * q + e];
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        int r, kk;
        amap(threadIdx.x + q * 256, r, kk);
        As[kk][r] = ra[q];
      }
    }
    if (VB && vb) {
#pragma unroll
      for (int q = 0; q < LB / 4; ++q) {
        const int i = threadIdx.x + q * 256;
        int kk, cc;
        if (TB) { kk = (i % (KT / 4)) * 4; cc = i / (KT / 4); }
        else { kk = i / (BN / 4); cc = (i % (BN / 4)) * 4; }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (TB) Bs[kk + e][cc] = rb[4 * q + e];
          else Bs[kk][cc + e] = rb[4 * q + e];
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        int kk, cc;
        bmap(threadIdx.x + q * 256, kk, cc);
        Bs[kk][cc] = rb[q];
      }
    }
    __syncthreads();
    if (k0 + KT < ke) fetch(k0 + KT);
#pragma unroll
    for (int ks = 0; ks < KT; ks += 4) {
      float a[WM], b[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) a[i] = As[ks + g][(wm * WM + i) * 16 + c];
#pragma unroll
      for (int j = 0; j < WN; ++j) b[j] = Bs[ks + g][(wn * WN + j) * 16 + c];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int gn = n0 + (wn * WN + j) * 16 + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + (wm * WM + i) * 16 + 4 * g + r;
        if (gm >= M || gn >= N) continue;
        float v = acc[i][j][r];
        if (EPI == EPI_BIAS || EPI == EPI_BIAS_RELU) v += bias[gn];
        if (EPI == EPI_BIAS_RELU) v = fmaxf(v, 0.f);
        if (EPI == EPI_MASK) v = mask[static_cast<int64_t>(gm) * ldm + gn] > 0.f ? v : 0.f;
        C[static_cast<int64_t>(gm) * ldc + gn] = v;
      }
    }
}

// A hidden layer of the BF16 forward pass on the matrix cores
// (v_mfma_f32_16x16x16bf16_1k): relu(A B + bias) with BF16 operands, FP32
// accumulation, bias and ReLU (A row-major M x K, B = the layer's FP32
// weights, row-major K x N).  A is FP32 (the features; rounded to BF16, to
// nearest even, on its way to LDS) or already BF16 (IN16: the first hidden
// layer's output).  OUT16: the result is stored as BF16.  FUSE: the result
// is not stored; instead each row's dot product with the output weights w3
// over the block's columns goes to ypart[(blockIdx.x * 2 + wave column) * M
// + row] (the output layer, summed by sum_parts_kernel).  Tiles, staging and
// prefetch as in gemm_mfma_kernel; LDS holds k contiguous per row of A and
// per column of B, so that lane l = 16 g + c reads its 4 operands
// A[i = c][k = 4g .. 4g+3] and B[k = 4g .. 4g+3][n = c] as one 8-byte word;
// its result register r holds D[i = 4 g + r][n = c].
typedef short mlp_s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short to_bf16(float x) {
  return __builtin_bit_cast(unsigned short, static_cast<__bf16>(x));
}

template <int WM, int WN, bool IN16, bool OUT16, bool FUSE>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K,
                                                        const void* __restrict__ Av, int lda,
                                                        const float* __restrict__ B, int ldb,
                                                        void* __restrict__ Cv, int ldc,
                                                        const float* __restrict__ bias,
                                                        const float* __restrict__ w3,
                                                        float* __restrict__ ypart) {
  constexpr int BM = 32 * WM, BN = 32 * WN, KT = 16, KP = KT + 4;   // KP: padded k stride
  constexpr int LA = BM * KT / 256, LB = KT * BN / 256;
  __shared__ __align__(16) unsigned short As[BM][KP];
  __shared__ __align__(16) unsigned short Bs[BN][KP];
  const float* A32 = static_cast<const float*>(Av);
  const unsigned short* A16 = static_cast<const unsigned short*>(Av);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int wm = wv >> 1, wn = wv & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  mlp_f4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = mlp_f4{0.f, 0.f, 0.f, 0.f};
  float ra[LA], rb[LB];
  unsigned short ra16[LA];
  auto fetch = [&](int k0) {
    const bool ka = k0 + KT <= K;
    if (ka && m0 + BM <= M) {
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        const int i = threadIdx.x + q * 256;
        const int64_t e = static_cast<int64_t>(m0 + i / KT) * lda + k0 + i % KT;
        if (IN16) ra16[q] = A16[e];
        else ra[q] = A32[e];
      }
    } else {
#pragma unroll
      for (int q = 0; q < LA; ++q) {
        const int i = threadIdx.x + q * 256;
        const int gm = m0 + i / KT, gk = k0 + i % KT;
        const bool in = gm < M && gk < K;
        const int64_t e = static_cast<int64_t>(gm) * lda + gk;
        if (IN16) ra16[q] = in ? A16[e] : static_cast<unsigned short>(0);
        else ra[q] = in ? A32[e] : 0.f;
      }
    }
    if (ka && n0 + BN <= N) {
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int i = threadIdx.x + q * 256;
        rb[q] = B[static_cast<int64_t>(k0 + i / BN) * ldb + n0 + i % BN];
      }
    } else {
#pragma unroll
      for (int q = 0; q < LB; ++q) {
        const int i = threadIdx.x + q * 256;
        const int gk = k0 + i / BN, gn = n0 + i % BN;
        rb[q] = (gk < K && gn < N) ? B[static_cast<int64_t>(gk) * ldb + gn] : 0.f;
      }
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += KT) {
#pragma unroll
    for (int q = 0; q < LA; ++q) {
      const int i = threadIdx.x + q * 256;
      As[i / KT][i % KT] = IN16 ? ra16[q] : to_bf16(ra[q]);
    }
#pragma unroll
    for (int q = 0; q < LB; ++q) {
      const int i = threadIdx.x + q * 256;
      Bs[i % BN][i / BN] = to_bf16(rb[q]);
    }
    __syncthreads();
    if (k0 + KT < K) fetch(k0 + KT);
    mlp_s4 a[WM], b[WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
      a[i] = *reinterpret_cast<const mlp_s4*>(&As[(wm * WM + i) * 16 + c][4 * g]);
#pragma unroll
    for (int j = 0; j < WN; ++j)
      b[j] = *reinterpret_cast<const mlp_s4*>(&Bs[(wn * WN + j) * 16 + c][4 * g]);
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int j = 0; j < WN; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  if (FUSE) {
    // rows 4g + r of tile i: dot with w3 over this lane's columns, then over
    // the 16 lanes of the group (xor 1 .. 8 stays inside the group)
    float part[WM][4];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) part[i][r] = 0.f;
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int gn = n0 + (wn * WN + j) * 16 + c;
      if (gn >= N) continue;
      const float bn = bias[gn], wo = w3[gn];
#pragma unroll
      for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) part[i][r] = fmaf(fmaxf(acc[i][j][r] + bn, 0.f), wo, part[i][r]);
    }
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = part[i][r];
#pragma unroll
        for (int off = 1; off < 16; off <<= 1) v += __shfl_xor(v, off);
        const int gm = m0 + (wm * WM + i) * 16 + 4 * g + r;
        if (c == 0 && gm < M) ypart[static_cast<int64_t>(blockIdx.x * 2 + wn) * M + gm] = v;
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int gn = n0 + (wn * WN + j) * 16 + c;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + (wm * WM + i) * 16 + 4 * g + r;
        if (gm >= M || gn >= N) continue;
        const float v = fmaxf(acc[i][j][r] + bias[gn], 0.f);
        const int64_t e = static_cast<int64_t>(gm) * ldc + gn;
        if (OUT16) static_cast<unsigned short*>(Cv)[e] = to_bf16(v);
        else static_cast<float*>(Cv)[e] = v;
      }
    }
}

// y[i] = b + sum over p < np of part[p * M + i], p in increasing order.
__global__ __launch_bounds__(256) void sum_parts_kernel(const float* part, int np, int M,
                                                        const float* b, float* y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= M) return;
  float s = 0.f;
  for (int p = 0; p < np; ++p) s += part[static_cast<int64_t>(p) * M + i];
  y[i] = s + b[0];
}

// y[i] = A[i, :] w + b (the output layer, N = 1): one wave per row, each
// lane a 16-byte piece of the row (rows 16-byte aligned, K % 4 == 0), then a
// butterfly sum across the wave.
// y[i] = A[i, :] . w + b; with t given also dy[i] = dscale (y[i] - t[i]), the
// gradient of the mean squared error (fused into the output layer when the
// training step does not report its loss).
__global__ __launch_bounds__(256) void gemv_bias_kernel(int M, int K, const float* __restrict__ A,
                                                        int lda, const float* __restrict__ w,
                                                        const float* __restrict__ b,
                                                        float* __restrict__ y,
                                                        const float* __restrict__ t = nullptr,
                                                        float* __restrict__ dy = nullptr,
                                                        float dscale = 0.f) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * 4;
  for (int i = blockIdx.x * 4 + (threadIdx.x >> 6); i < M; i += nw) {
    const float* row = A + static_cast<int64_t>(i) * lda;
    float acc = 0.f;
    for (int k = lane * 4; k < K; k += 256) {
      const float4 a = *reinterpret_cast<const float4*>(row + k);
      acc = fmaf(a.x, w[k], acc);
      acc = fmaf(a.y, w[k + 1], acc);
      acc = fmaf(a.z, w[k + 2], acc);
      acc = fmaf(a.w, w[k + 3], acc);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) {
      const float yi = acc + b[0];
      y[i] = yi;
      if (t) dy[i] = dscale * (yi - t[i]);
    }
  }
}

// Column sums of D [rows][N], each row weighted by wr[row] when wr is not
// null (the bias gradients, and the output layer's weight gradient
// H2^T dy), in two fixed-order stages.  Stage 1, N = 256 (colsum4_kernel):
// block y sums rows [y rc, (y + 1) rc) of every column; lane l of each of its
// 16 waves owns columns 4l .. 4l+3 (one 16-byte load per row), wave w takes
// rows r0 + w + 16i with four rows in flight, and the wave sums are added in
// wave order into part[y * N + column].  N = 1 (colsum1_kernel): every thread
// of block y sums rows r0 + t + 256 i in order, then the block's threads in
// a fixed tree.  Stage 2: split_sum_kernel adds the row chunks in order.
constexpr int kColsumWaves = 16;
__global__ __launch_bounds__(64 * kColsumWaves) void colsum4_kernel(const float* D, const float* wr,
                                                                    int rows, int rc, float* part) {
  constexpr int NW = kColsumWaves;
  __shared__ float4 ws[NW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r0 = blockIdx.y * rc, r1 = min(rows, r0 + rc);
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  const float4* D4 = reinterpret_cast<const float4*>(D) + lane;
  auto add = [&](int r) {
    const float4 d = D4[static_cast<int64_t>(r) * 64];
    if (wr) {
      const float q = wr[r];
      s.x = fmaf(d.x, q, s.x);
      s.y = fmaf(d.y, q, s.y);
      s.z = fmaf(d.z, q, s.z);
      s.w = fmaf(d.w, q, s.w);
    } else {
      s.x += d.x;
      s.y += d.y;
      s.z += d.z;
      s.w += d.w;
    }
  };
  int r = r0 + w;
  for (; r + 3 * NW < r1; r += 4 * NW) {      // four rows of this wave in flight
    add(r);
    add(r + NW);
    add(r + 2 * NW);
    add(r + 3 * NW);
  }
  for (; r < r1; r += NW) add(r);
  ws[w][lane] = s;
  __syncthreads();
  if (w == 0) {
    float4 t = ws[0][lane];
#pragma unroll
    for (int q = 1; q < NW; ++q) {
      t.x += ws[q][lane].x;
      t.y += ws[q][lane].y;
      t.z += ws[q][lane].z;
      t.w += ws[q][lane].w;
    }
    reinterpret_cast<float4*>(part + static_cast<int64_t>(blockIdx.y) * 256)[lane] = t;
  }
}

__global__ __launch_bounds__(256) void colsum1_kernel(const float* D, const float* wr, int rows,
                                                      int rc, float* part) {
  __shared__ float red[256];
  const int r0 = blockIdx.y * rc, r1 = min(rows, r0 + rc);
  float s = 0.f;
  for (int r = r0 + threadIdx.x; r < r1; r += 256) s = wr ? fmaf(D[r], wr[r], s) : s + D[r];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y] = red[0];
}

// C[i] = sum over z < ks of P[z * len + i], z in increasing order.
__global__ __launch_bounds__(256) void split_sum_kernel(const float* P, int ks, int len, float* C) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= len) return;
  float s = 0.f;
#pragma unroll 8
  for (int z = 0; z < ks; ++z) s += P[static_cast<int64_t>(z) * len + i];   // loads ahead, adds in order
  C[i] = s;
}

constexpr int kSplitMax = 32;          // K slices of a split product
constexpr int kSplitWords = kSplitMax * kH * kH;
constexpr int kColsumChunks = 64;      // row chunks of a column sum (<= kSplitWords / kH)

// Products with few output tiles and a long K (the weight and bias
// gradients, K = batch) are split over K into slices of at most 512 blocks
// in all (two per CU), the partials (in part, kSplitWords floats) summed in
// slice order.
template <bool TA, bool TB, int EPI>
static void gemm(int M, int N, int K, const float* A, int lda, const float* B, int ldb, float* C,
                 int ldc, const float* bias, const float* mask, int ldm, hipStream_t st,
                 float* part = nullptr) {
  if (!TA && !TB && EPI == EPI_BIAS && N == 1 && ldb == 1 && K % 4 == 0 && lda % 4 == 0 &&
      (reinterpret_cast<uintptr_t>(A) & 15) == 0) {
    const int blocks = std::min((M + 3) / 4, 8192);
    hipLaunchKernelGGL(gemv_bias_kernel, dim3(blocks), dim3(256), 0, st, M, K, A, lda, B, bias, C);
    return;
  }
  // matrix cores for every product with at least 64 rows, 64 columns and a
  // 16-deep k (128 x 128 tiles for the large forward products, else 64 x 64);
  // the rest (bias gradients, rank-1 updates) on the vector tile kernel
  const bool mfma = M >= 64 && N >= 64 && K >= 16;
  const bool big = mfma && !TA && M >= 32768;
  const int TM = big ? 128 : 64, TN = big ? 128 : 64;
  const int tiles = ((N + TN - 1) / TN) * ((M + TM - 1) / TM);
  int ks = 1;
  if (EPI == EPI_NONE && part && tiles < 64 && K >= 2048 && ldc == N) {
    ks = 512 / tiles;
    if (ks > kSplitMax) ks = kSplitMax;
    if (ks > K / 128) ks = K / 128;
    if (static_cast<int64_t>(ks) * M * N > kSplitWords) ks = static_cast<int>(kSplitWords / (M * N));
  }
  // 16-byte slice loads for each operand that allows them (not the 130-wide
  // feature rows)
  const bool va = lda % 4 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0;
  const bool vb = ldb % 4 == 0 && (reinterpret_cast<uintptr_t>(B) & 15) == 0;
  auto launch = [&](dim3 grid, float* out, int ldo, int kc) {
#define CPM_GEMM_MFMA(W, VA_, VB_)                                                            \
  hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, W, W, EPI, VA_, VB_>), grid, dim3(256), 0, st, M, N, \
                     K, A, lda, B, ldb, out, ldo, bias, mask, ldm, kc)
    if (big) {
      if (va && vb) CPM_GEMM_MFMA(4, true, true);
      else if (vb) CPM_GEMM_MFMA(4, false, true);
      else if (va) CPM_GEMM_MFMA(4, true, false);
      else CPM_GEMM_MFMA(4, false, false);
    } else if (mfma) {
      if (va && vb) CPM_GEMM_MFMA(2, true, true);
      else if (vb) CPM_GEMM_MFMA(2, false, true);
      else if (va) CPM_GEMM_MFMA(2, true, false);
      else CPM_GEMM_MFMA(2, false, false);
    } else {
      hipLaunchKernelGGL((gemm_kernel<TA, TB, EPI>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb,
                         out, ldo, bias, mask, ldm, kc);
    }
  };
#undef CPM_GEMM_MFMA
  if (ks <= 1) {
    launch(dim3((N + TN - 1) / TN, (M + TM - 1) / TM), C, ldc, K);
    return;
  }
  const int kc = ((K + ks - 1) / ks + 15) & ~15;
  ks = (K + kc - 1) / kc;
  launch(dim3((N + TN - 1) / TN, (M + TM - 1) / TM, ks), part, N, kc);
  const int len = M * N;
  hipLaunchKernelGGL(split_sum_kernel, dim3((len + 255) / 256), dim3(256), 0, st,
                     static_cast<const float*>(part), ks, len, C);
}

static int feature_blocks(int rows) {
  return static_cast<int>(std::min<int64_t>((static_cast<int64_t>(rows) * kF + 255) / 256, 16384));
}

// db [N] = column sums of D [rows][N], rows weighted by wr if not null
// (part: kSplitWords floats).
static void colsum(const float* D, const float* wr, int rows, int N, float* db, float* part,
                   hipStream_t st) {
  // N is 256 (the hidden layers; D 16-byte aligned) or 1 (the output layer)
  int ks = std::max(1, std::min(kColsumChunks, rows / 256));
  const int rc = (rows + ks - 1) / ks;
  ks = (rows + rc - 1) / rc;
  if (N == kH)
    hipLaunchKernelGGL(colsum4_kernel, dim3(1, ks), dim3(64 * kColsumWaves), 0, st, D, wr, rows, rc,
                       part);
  else
    hipLaunchKernelGGL(colsum1_kernel, dim3(1, ks), dim3(256), 0, st, D, wr, rows, rc, part);
  hipLaunchKernelGGL(split_sum_kernel, dim3((N + 255) / 256), dim3(256), 0, st,
                     static_cast<const float*>(part), ks, N, db);
}

// -------------------------------------------------------------- features
// Row i of X for state s of an m^3 grid:
//   [0..2]    i_k / (m - 1)
//   [3..127]  10 * R(clamp(i + d)) for d in {-2..2}^3, d_0 slowest
//   [128]     (gamma - 0.945) / 0.026
//   [129]     (slip - 0.175) / 0.072
// computed one feature at a time.
__device__ __forceinline__ float feature_at(const float* R, int m, FastDiv dm, float gamma,
                                            float slip, int s, int f) {
  const uint32_t q1 = fdiv(static_cast<uint32_t>(s), dm), q2 = fdiv(q1, dm);
  const int i2 = s - static_cast<int>(q1) * m, i1 = static_cast<int>(q1 - q2 * m),
            i0 = static_cast<int>(q2);
  if (f < 3) {
    const float inv = m > 1 ? 1.0f / static_cast<float>(m - 1) : 0.f;
    return (f == 0 ? i0 : (f == 1 ? i1 : i2)) * inv;
  }
  if (f == 128) return (gamma - kGammaMean) * kGammaScale;
  if (f == 129) return (slip - kSlipMean) * kSlipScale;
  const int j = f - 3;
  const int j0 = min(max(i0 + j / 25 - 2, 0), m - 1);
  const int j1 = min(max(i1 + (j / 5) % 5 - 2, 0), m - 1);
  const int j2 = min(max(i2 + j % 5 - 2, 0), m - 1);
  return kRScale * R[(j0 * m + j1) * m + j2];
}

// All states s0 .. s0+count-1 of one instance, one thread per (state,
// feature): consecutive threads write consecutive words of a row of X (row
// stride ldx >= 130).  IDX is the word-index type (32-bit while
// count * ldx < 2^31).
template <typename IDX>
__global__ void features_range_kernel(const float* R, int m, FastDiv dm, float gamma, float slip,
                                      int s0, int count, float* X, int ldx) {
  const IDX total = static_cast<IDX>(count) * kF;
  const IDX stride = static_cast<IDX>(gridDim.x) * blockDim.x;
  for (IDX e = static_cast<IDX>(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    const IDX i = e / kF;
    const int f = static_cast<int>(e - i * kF);
    X[i * static_cast<IDX>(ldx) + f] = feature_at(R, m, dm, gamma, slip, s0 + static_cast<int>(i), f);
  }
}

static void launch_features_range(const float* R, int m, float gamma, float slip, int s0, int count,
                                  float* X, int ldx, hipStream_t st) {
  const FastDiv dm = make_fastdiv(static_cast<uint32_t>(m));
  const int blocks = feature_blocks(count);
  if (static_cast<int64_t>(count) * ldx < (int64_t{1} << 31))
    hipLaunchKernelGGL(features_range_kernel<uint32_t>, dim3(blocks), dim3(256), 0, st, R, m, dm,
                       gamma, slip, s0, count, X, ldx);
  else
    hipLaunchKernelGGL(features_range_kernel<int64_t>, dim3(blocks), dim3(256), 0, st, R, m, dm,
                       gamma, slip, s0, count, X, ldx);
}

// n states spread evenly over an instance of S states: sample j is state
// floor(j S / n); one thread per (sample, feature); rows of kXS words.
__global__ void features_spread_kernel(const float* R, int m, FastDiv dm, float gamma, float slip,
                                       int S, int n, float* X) {
  const int64_t total = static_cast<int64_t>(n) * kF;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total; e += stride) {
    const int64_t j = e / kF;
    const int st = static_cast<int>(j * S / n);
    const int f = static_cast<int>(e - j * kF);
    X[j * kXS + f] = feature_at(R, m, dm, gamma, slip, st, f);
  }
}

// Minibatch: sample i -> (instance, state) drawn with SplitMix64 from
// (seed, step, i); features and the target (1 - gamma) V*(s).
// One thread per (sample, feature), rows of kXS words; every thread of a
// sample draws the same (instance, state), the feature-0 thread also writes
// the target.
__global__ void features_sample_kernel(const float* const* R_ptrs, const double* const* V_ptrs,
                                       const double* gammas, const double* slips, int n_inst,
                                       int m, FastDiv dm, uint64_t seed, int64_t step, int count,
                                       float* X, float* t, double* loss) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *loss = 0.0;   // the step's loss accumulates later
  const int64_t total = static_cast<int64_t>(count) * kF;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  const int S = m * m * m;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total; e += stride) {
    const int i = static_cast<int>(e / kF), f = static_cast<int>(e - static_cast<int64_t>(i) * kF);
    const uint64_t r = splitmix64(seed ^ splitmix64(static_cast<uint64_t>(step) * 0x100000001B3ull +
                                                    static_cast<uint64_t>(i)));
    const int inst = static_cast<int>((r >> 32) % static_cast<uint64_t>(n_inst));
    const int s = static_cast<int>((r & 0xFFFFFFFFull) % static_cast<uint64_t>(S));
    X[static_cast<int64_t>(i) * kXS + f] = feature_at(R_ptrs[inst], m, dm, static_cast<float>(gammas[inst]),
                                                      static_cast<float>(slips[inst]), s, f);
    if (f == 0)
      t[i] = static_cast<float>(((1.0 - gammas[inst]) * V_ptrs[inst][s] - kOutMean) / kOutScale);
  }
}

// -------------------------------------------------------------- loss, misc
__global__ void mse_kernel(const float* y, const float* t, int count, float* dy, double* loss) {
  __shared__ double part[4];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double l = 0.0;
  if (i < count) {
    const float d = y[i] - t[i];
    dy[i] = 2.0f * d / static_cast<float>(count);
    l = static_cast<double>(d) * d / count;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) l += __shfl_xor(l, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(loss, part[0] + part[1] + part[2] + part[3]);
}

__global__ void fill_kernel(float* p, int64_t n, float v) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void adam_kernel(float* p, float* m, float* v, const float* g, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// He-normal hidden weights (std sqrt(2 / fan_in)); zero biases and a zero
// output layer, so training starts from the constant prediction kOutMean.
__global__ void init_kernel(float* p, uint64_t seed) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= kParams) return;
  float fan_in = 0.f;
  if (i < kOffB1) fan_in = kF;
  else if (i >= kOffW2 && i < kOffB2) fan_in = kH;
  if (fan_in == 0.f) {
    p[i] = 0.f;
    return;
  }
  const uint64_t r1 = splitmix64(seed ^ splitmix64(2 * static_cast<uint64_t>(i)));
  const uint64_t r2 = splitmix64(seed ^ splitmix64(2 * static_cast<uint64_t>(i) + 1));
  const float z = sqrtf(-2.f * logf(u01(r1))) * cosf(6.2831853f * u01(r2));
  p[i] = z * sqrtf(2.f / fan_in);
}

__global__ void to_values_kernel(const float* y, int count, double inv_scale, double* V) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) V[i] = (kOutMean + kOutScale * static_cast<double>(y[i])) * inv_scale;
}

// Level of a prediction: the mean of the network's values over n sampled
// states (the outputs y of one forward pass), summed in a fixed order
// (kLevelBlocks strided partial sums, then the partials in order by every
// block of the fill kernel), so repeated predictions agree bit for bit; then
// every entry of V is set to it.
constexpr int kLevelBlocks = 16;
constexpr int kLevelSamples = 4096;

__global__ __launch_bounds__(256) void level_partial_kernel(const float* y, int n, double* part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    acc += kOutMean + kOutScale * static_cast<double>(y[i]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void level_fill_kernel(double* V, int64_t S, const double* part,
                                                         int nparts, int n, double inv_scale) {
  double tot = 0.0;
  for (int b = 0; b < nparts; ++b) tot += part[b];     // same order in every thread
  const double level = tot / static_cast<double>(n) * inv_scale;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(256) + threadIdx.x; i < S;
       i += static_cast<int64_t>(gridDim.x) * 256)
    V[i] = level;
}

// ----------------------------------------------------------- workspace
struct MlpWs {
  float *X, *H1, *H2, *y, *t, *dy, *dH1, *dH2;
  double* loss;
  float* part;                      // split-K partials (dW2, on the side stream in training)
  float* part2;                     // column-sum partials (the side stream's)
  float* part3;                     // split-K partials of dW1 (the caller's stream)
};

static constexpr size_t al(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

constexpr size_t mlp_ws_bytes(int B) {
  const size_t b = static_cast<size_t>(B);
  return al(b * kXS * 4) + 4 * al(b * kH * 4) + 3 * al(b * 4) + al(b * 4) + al(64) +
         al(static_cast<size_t>(kSplitWords) * 4) + al(static_cast<size_t>(kColsumChunks) * kH * 4) +
         al(static_cast<size_t>(kSplitMax) * kF * kH * 4);
}

MlpWs carve(void* ws, int B) {
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t sz) {
    char* q = p;
    p += al(sz);
    return q;
  };
  const size_t b = static_cast<size_t>(B);
  MlpWs w{};
  w.X = reinterpret_cast<float*>(take(b * kXS * 4));
  w.H1 = reinterpret_cast<float*>(take(b * kH * 4));
  w.H2 = reinterpret_cast<float*>(take(b * kH * 4));
  w.dH1 = reinterpret_cast<float*>(take(b * kH * 4));
  w.dH2 = reinterpret_cast<float*>(take(b * kH * 4));
  w.y = reinterpret_cast<float*>(take(b * 4));
  w.t = reinterpret_cast<float*>(take(b * 4));
  w.dy = reinterpret_cast<float*>(take(b * 4));
  w.loss = reinterpret_cast<double*>(take(64));
  w.part = reinterpret_cast<float*>(take(static_cast<size_t>(kSplitWords) * 4));
  w.part2 = reinterpret_cast<float*>(take(static_cast<size_t>(kColsumChunks) * kH * 4));
  w.part3 = reinterpret_cast<float*>(take(static_cast<size_t>(kSplitMax) * kF * kH * 4));
  return w;
}

// BF16 forward pass: first hidden layer stored as BF16 (in H1's space), the
// second fused with the output layer (row partials in H2's space).
static void forward_bf16(const float* P, const float* X, int ldx, int M, const MlpWs& w,
                         hipStream_t st) {
  float* ypart = w.H2;
  if (M >= 32768) {
    const dim3 grid(kH / 128, (M + 127) / 128);
    hipLaunchKernelGGL((gemm_bf16_kernel<4, 4, false, true, false>), grid, dim3(256), 0, st, M, kH,
                       kF, static_cast<const void*>(X), ldx, P + kOffW1, kH, static_cast<void*>(w.H1),
                       kH, P + kOffB1, nullptr, nullptr);
    hipLaunchKernelGGL((gemm_bf16_kernel<4, 4, true, false, true>), grid, dim3(256), 0, st, M, kH,
                       kH, static_cast<const void*>(w.H1), kH, P + kOffW2, kH, nullptr, 0, P + kOffB2,
                       P + kOffW3, ypart);
  } else {
    const dim3 grid(kH / 64, (M + 63) / 64);
    hipLaunchKernelGGL((gemm_bf16_kernel<2, 2, false, true, false>), grid, dim3(256), 0, st, M, kH,
                       kF, static_cast<const void*>(X), ldx, P + kOffW1, kH, static_cast<void*>(w.H1),
                       kH, P + kOffB1, nullptr, nullptr);
    hipLaunchKernelGGL((gemm_bf16_kernel<2, 2, true, false, true>), grid, dim3(256), 0, st, M, kH,
                       kH, static_cast<const void*>(w.H1), kH, P + kOffW2, kH, nullptr, 0, P + kOffB2,
                       P + kOffW3, ypart);
  }
  const int np = 2 * (M >= 32768 ? kH / 128 : kH / 64);
  hipLaunchKernelGGL(sum_parts_kernel, dim3((M + 255) / 256), dim3(256), 0, st,
                     static_cast<const float*>(ypart), np, M, P + kOffB3, w.y);
}

// with_dy: the output layer also writes dy, the loss gradient against w.t
// (training steps whose loss is not read)
// X: rows of ldx words (kXS for the workspace's own features, kF for a
// caller's X [B][130]).
void forward(const float* P, const float* X, int ldx, int B, const MlpWs& w, hipStream_t st,
             bool bf16, bool with_dy = false) {
  if (bf16) {
    forward_bf16(P, X, ldx, B, w, st);
    return;
  }
  gemm<false, false, EPI_BIAS_RELU>(B, kH, kF, X, ldx, P + kOffW1, kH, w.H1, kH, P + kOffB1, nullptr, 0, st);
  gemm<false, false, EPI_BIAS_RELU>(B, kH, kH, w.H1, kH, P + kOffW2, kH, w.H2, kH, P + kOffB2, nullptr, 0, st);
  if (with_dy) {
    const int blocks = std::min((B + 3) / 4, 8192);
    hipLaunchKernelGGL(gemv_bias_kernel, dim3(blocks), dim3(256), 0, st, B, kH,
                       static_cast<const float*>(w.H2), kH, P + kOffW3, P + kOffB3, w.y,
                       static_cast<const float*>(w.t), w.dy, 2.0f / static_cast<float>(B));
    return;
  }
  gemm<false, false, EPI_BIAS>(B, 1, kH, w.H2, kH, P + kOffW3, 1, w.y, 1, P + kOffB3, nullptr, 0, st);
}

// dH2 = (dy w3^T) .* [H2 > 0]: the output layer's input gradient, a rank-1
// product masked by the ReLU, as an elementwise pass over H2 (four columns
// per thread, 16-byte loads and stores).
__global__ __launch_bounds__(256) void rank1_mask_kernel(const float* __restrict__ dy,
                                                         const float* __restrict__ w3,
                                                         const float* __restrict__ H2, int rows,
                                                         float* __restrict__ dH2) {
  const int64_t total = static_cast<int64_t>(rows) * (kH / 4);
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total; e += stride) {
    const int64_t r = e / (kH / 4);
    const int c4 = static_cast<int>(e - r * (kH / 4));
    const float d = dy[r];
    const float4 h = reinterpret_cast<const float4*>(H2)[e];
    const float4 w = reinterpret_cast<const float4*>(w3)[c4];
    float4 o;
    o.x = h.x > 0.f ? d * w.x : 0.f;
    o.y = h.y > 0.f ? d * w.y : 0.f;
    o.z = h.z > 0.f ? d * w.z : 0.f;
    o.w = h.w > 0.f ? d * w.w : 0.f;
    reinterpret_cast<float4*>(dH2)[e] = o;
  }
}

// Second stream of the backward pass, one per device (default priority, like
// every stream here): the column sums run there beside the products.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t ev[4] = {};
};
constexpr int kMaxSideDevices = 64;
std::mutex g_side_mu;
SideStream g_side[kMaxSideDevices];

// The current device's side stream, created on first use; nullptr if it
// cannot be had (the caller then runs everything on its own stream).
SideStream* side_stream() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxSideDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_side_mu);
  SideStream& ss = g_side[dev];
  if (!ss.s) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    for (auto& e : ss.ev)
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    ss.s = s;
  }
  return &ss;
}

// Gradient of the mean squared error (y - t)^2 over the B rows of X.  The
// column sums (dw3, db3, db2, db1) read activations that are final once the
// products before them have run, so they go to the side stream, forked and
// joined with events, with their own partial area; so does dW2 = H1^T dH2,
// which needs only dH2 and runs beside the product for dH1 (each split-K
// product has its own partial area).  The same kernels in the same order per
// stream: the result does not depend on how the two streams interleave.
// have_dy: the forward pass already wrote dy (and the loss is not wanted).
void backward(const float* P, const float* X, int ldx, int B, const MlpWs& w, float* G, hipStream_t st,
              bool have_dy = false) {
  const int nb = (B + 255) / 256;
  if (!have_dy)
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, st, w.y, w.t, B, w.dy, w.loss);
  SideStream* ss = side_stream();
  const hipStream_t so = ss ? ss->s : st;
  auto fork = [&](int i) {
    if (!ss) return;
    (void)hipEventRecord(ss->ev[i], st);
    (void)hipStreamWaitEvent(so, ss->ev[i], 0);
  };
  // layer 3: dw3 = H2^T dy, db3 = 1^T dy, dH2 = (dy w3^T) .* [H2 > 0]
  fork(0);
  colsum(w.H2, w.dy, B, kH, G + kOffW3, w.part2, so);
  colsum(w.dy, nullptr, B, 1, G + kOffB3, w.part2, so);
  hipLaunchKernelGGL(rank1_mask_kernel,
                     dim3(static_cast<unsigned>(std::min<int64_t>(
                         (static_cast<int64_t>(B) * (kH / 4) + 255) / 256, 8192))),
                     dim3(256), 0, st, w.dy, P + kOffW3, w.H2, B, w.dH2);
  // layer 2: dW2 = H1^T dH2, db2 = 1^T dH2, dH1 = (dH2 W2^T) .* [H1 > 0]
  fork(1);
  colsum(w.dH2, nullptr, B, kH, G + kOffB2, w.part2, so);
  gemm<true, false, EPI_NONE>(kH, kH, B, w.H1, kH, w.dH2, kH, G + kOffW2, kH, nullptr, nullptr, 0, so, w.part);
  gemm<false, true, EPI_MASK>(B, kH, kH, w.dH2, kH, P + kOffW2, kH, w.dH1, kH, nullptr, w.H1, kH, st);
  // layer 1: dW1 = X^T dH1, db1 = 1^T dH1
  fork(2);
  colsum(w.dH1, nullptr, B, kH, G + kOffB1, w.part2, so);
  gemm<true, false, EPI_NONE>(kF, kH, B, X, ldx, w.dH1, kH, G + kOffW1, kH, nullptr, nullptr, 0, st, w.part3);
  if (ss) {   // join: the caller's stream waits for the side stream's sums
    (void)hipEventRecord(ss->ev[3], so);
    (void)hipStreamWaitEvent(st, ss->ev[3], 0);
  }
}

int mfail(const std::string& m) { return fail(nullptr, CPMDP_E_ARG, m); }

// Scratch of the allocation-free prediction (cpmdp_mlp_predict_noalloc):
// the MLP workspace for chunks of up to kStaticRows rows, 30.3 MiB, held by
// every GPU the library runs on until the process ends.  Host code never
// passes `scratch` itself (its host-side name is no device address): the
// device address comes from hipGetSymbolAddress, once per device.
constexpr int kStaticRows = 4096;
constexpr size_t kStaticBytes = mlp_ws_bytes(kStaticRows);
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of the current device's scratch (looked up on the first
// call on that device, with that device current).
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices)
    return fail(nullptr, CPMDP_E_DEVICE, "no current device for the static scratch");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(nullptr, CPMDP_E_DEVICE,
                  std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CPMDP_OK;
}

}  // namespace cpm

using namespace cpm;

extern "C" {

int cpmdp_mlp_param_count(int64_t* count) {
  if (!count) return mfail("count is NULL");
  *count = kParams;
  return CPMDP_OK;
}

int cpmdp_mlp_workspace_bytes(int32_t batch, size_t* bytes) {
  if (!bytes || batch < 1) return mfail("batch >= 1 and bytes non-NULL");
  *bytes = mlp_ws_bytes(batch);
  return CPMDP_OK;
}

int cpmdp_mlp_init(float* params, uint64_t seed, void* stream) {
  if (!params) return mfail("params is NULL");
  hipLaunchKernelGGL(init_kernel, dim3((kParams + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(stream), params, seed);
  return hipGetLastError() == hipSuccess ? CPMDP_OK : fail(nullptr, CPMDP_E_DEVICE, "init launch");
}

int cpmdp_mlp_features(const float* R, int32_t m, double gamma, double slip, int32_t s0,
                       int32_t count, float* X, void* stream) {
  if (!R || !X || m < 1 || count < 0 || s0 < 0 ||
      static_cast<int64_t>(m) * m * m >= (int64_t{1} << 31) ||
      static_cast<int64_t>(s0) + count > static_cast<int64_t>(m) * m * m)
    return mfail("bad feature arguments");
  if (count == 0) return CPMDP_OK;
  launch_features_range(R, m, static_cast<float>(gamma), static_cast<float>(slip), s0, count, X, kF,
                        static_cast<hipStream_t>(stream));
  return hipGetLastError() == hipSuccess ? CPMDP_OK : fail(nullptr, CPMDP_E_DEVICE, "features launch");
}

int cpmdp_mlp_forward(const float* params, const float* X, int32_t count, float* y,
                      int32_t precision, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !X || !y || !ws || count < 1) return mfail("bad forward arguments");
  if (precision != CPMDP_FP32 && precision != CPMDP_BF16)
    return mfail("precision must be CPMDP_FP32 or CPMDP_BF16");
  if (ws_bytes < mlp_ws_bytes(count)) return fail(nullptr, CPMDP_E_WORKSPACE, "MLP workspace too small");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  MlpWs w = carve(ws, count);
  forward(params, X, kF, count, w, st, precision == CPMDP_BF16);
  (void)hipMemcpyAsync(y, w.y, count * 4, hipMemcpyDeviceToDevice, st);
  return hipGetLastError() == hipSuccess ? CPMDP_OK : fail(nullptr, CPMDP_E_DEVICE, "forward launch");
}

int cpmdp_mlp_loss_grad(const float* params, const float* X, const float* t, int32_t count,
                        float* grad, double* loss_out, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !X || !t || !grad || !ws || count < 1) return mfail("bad loss_grad arguments");
  if (ws_bytes < mlp_ws_bytes(count)) return fail(nullptr, CPMDP_E_WORKSPACE, "MLP workspace too small");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  MlpWs w = carve(ws, count);
  (void)hipMemcpyAsync(w.t, t, count * 4, hipMemcpyDeviceToDevice, st);
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<float*>(w.loss), 2, 0.0f);
  forward(params, X, kF, count, w, st, false);
  backward(params, X, kF, count, w, grad, st);
  if (hipGetLastError() != hipSuccess) return fail(nullptr, CPMDP_E_DEVICE, "loss_grad launch");
  if (loss_out) {
    if (hipMemcpyAsync(loss_out, w.loss, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(nullptr, CPMDP_E_DEVICE, "loss read");
  }
  return CPMDP_OK;
}

int cpmdp_mlp_adam(float* params, float* m, float* v, const float* grad, int64_t step, double lr,
                   void* stream) {
  if (!params || !m || !v || !grad || step < 1 || !(lr > 0)) return mfail("bad adam arguments");
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, static_cast<float>(step));
  const float c2 = 1.f - std::pow(b2, static_cast<float>(step));
  hipLaunchKernelGGL(adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0,
                     static_cast<hipStream_t>(stream), params, m, v, grad, kParams,
                     static_cast<float>(lr), b1, b2, 1e-8f, c1, c2);
  return hipGetLastError() == hipSuccess ? CPMDP_OK : fail(nullptr, CPMDP_E_DEVICE, "adam launch");
}

int cpmdp_mlp_train_step(float* params, float* adam_m, float* adam_v, float* grad, int64_t step,
                         const float* const* R_ptrs, const double* const* Vstar_ptrs,
                         const double* gammas, const double* slips, int32_t n_inst, int32_t m,
                         int32_t batch, uint64_t seed, double lr, void* ws, size_t ws_bytes,
                         void* stream, double* loss_out) {
  if (!params || !adam_m || !adam_v || !grad || !R_ptrs || !Vstar_ptrs || !gammas || !slips ||
      n_inst < 1 || m < 1 || batch < 1 || step < 1 || !ws)
    return mfail("bad train_step arguments");
  if (static_cast<int64_t>(m) * m * m >= (int64_t{1} << 31))
    return mfail("train_step: m^3 must be below 2^31");
  if (ws_bytes < mlp_ws_bytes(batch)) return fail(nullptr, CPMDP_E_WORKSPACE, "MLP workspace too small");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  MlpWs w = carve(ws, batch);
  hipLaunchKernelGGL(features_sample_kernel, dim3(feature_blocks(batch)), dim3(256), 0, st, R_ptrs,
                     Vstar_ptrs, gammas, slips, n_inst, m, make_fastdiv(static_cast<uint32_t>(m)),
                     seed, step, batch, w.X, w.t, w.loss);
  // without a loss to report, the output layer writes the loss gradient too
  forward(params, w.X, kXS, batch, w, st, false, loss_out == nullptr);
  backward(params, w.X, kXS, batch, w, grad, st, loss_out == nullptr);
  int rc = cpmdp_mlp_adam(params, adam_m, adam_v, grad, step, lr, stream);
  if (rc) return rc;
  if (hipGetLastError() != hipSuccess) return fail(nullptr, CPMDP_E_DEVICE, "train_step launch");
  if (loss_out) {
    if (hipMemcpyAsync(loss_out, w.loss, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(nullptr, CPMDP_E_DEVICE, "loss read");
  }
  return CPMDP_OK;
}

int cpmdp_mlp_predict(const float* params, const float* R, int32_t m, double gamma, double slip,
                      double* V0, int32_t chunk, int32_t precision, int32_t level, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!params || !R || !V0 || m < 1 || chunk < 1 || !ws || !(gamma < 1.0) ||
      (level != 0 && level != 1))
    return mfail("bad predict arguments");
  if (static_cast<int64_t>(m) * m * m >= (int64_t{1} << 31))
    return mfail("predict: m^3 must be below 2^31");
  if (precision != CPMDP_FP32 && precision != CPMDP_BF16)
    return mfail("precision must be CPMDP_FP32 or CPMDP_BF16");
  if (ws_bytes < mlp_ws_bytes(chunk)) return fail(nullptr, CPMDP_E_WORKSPACE, "MLP workspace too small");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int S = m * m * m;
  MlpWs w = carve(ws, chunk);
  if (level) {
    // the network on n states spread over the grid; V0 = their mean everywhere
    const int n = std::min(std::min(S, chunk), kLevelSamples);
    hipLaunchKernelGGL(features_spread_kernel, dim3(feature_blocks(n)), dim3(256), 0, st, R, m,
                       make_fastdiv(static_cast<uint32_t>(m)), static_cast<float>(gamma),
                       static_cast<float>(slip), S, n, w.X);
    forward(params, w.X, kXS, n, w, st, precision == CPMDP_BF16);
    // the split-K partial area is free once the forward pass is done
    double* part = reinterpret_cast<double*>(w.part);
    hipLaunchKernelGGL(level_partial_kernel, dim3(kLevelBlocks), dim3(256), 0, st, w.y, n, part);
    hipLaunchKernelGGL(level_fill_kernel, dim3(std::min(1024, (S + 255) / 256)), dim3(256), 0, st,
                       V0, static_cast<int64_t>(S), part, kLevelBlocks, n, 1.0 / (1.0 - gamma));
    return hipGetLastError() == hipSuccess ? CPMDP_OK
                                           : fail(nullptr, CPMDP_E_DEVICE, "predict launch");
  }
  for (int s0 = 0; s0 < S; s0 += chunk) {
    const int cnt = std::min(chunk, S - s0);
    launch_features_range(R, m, static_cast<float>(gamma), static_cast<float>(slip), s0, cnt, w.X,
                          kXS, st);
    forward(params, w.X, kXS, cnt, w, st, precision == CPMDP_BF16);
    hipLaunchKernelGGL(to_values_kernel, dim3((cnt + 255) / 256), dim3(256), 0, st, w.y, cnt,
                       1.0 / (1.0 - gamma), V0 + s0);
  }
  return hipGetLastError() == hipSuccess ? CPMDP_OK : fail(nullptr, CPMDP_E_DEVICE, "predict launch");
}

int cpmdp_mlp_predict_levels(const float* params, const float* const* R, const double* gammas,
                             const double* slips, int32_t n_inst, int32_t m, double* const* V0,
                             int32_t precision, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !R || !gammas || !slips || !V0 || n_inst < 1 || m < 1 || !ws)
    return mfail("bad predict_levels arguments");
  if (static_cast<int64_t>(m) * m * m >= (int64_t{1} << 31))
    return mfail("predict_levels: m^3 must be below 2^31");
  if (precision != CPMDP_FP32 && precision != CPMDP_BF16)
    return mfail("precision must be CPMDP_FP32 or CPMDP_BF16");
  const int S = m * m * m;
  const int n = std::min(S, kLevelSamples);
  // the rows of one forward pass, and each instance's kLevelBlocks partial
  // sums (FP64) in the split-K partial area
  if (static_cast<int64_t>(n) * n_inst > (int64_t{1} << 24) ||
      static_cast<int64_t>(n_inst) * kLevelBlocks * 2 > kSplitWords)
    return mfail("predict_levels: too many instances for one pass (n_inst * min(m^3, 4096) > 2^24)");
  for (int i = 0; i < n_inst; ++i)
    if (!R[i] || !V0[i] || !(gammas[i] < 1.0))
      return mfail("predict_levels: null R or V0, or gamma >= 1, for an instance");
  const int rows = n * n_inst;
  if (ws_bytes < mlp_ws_bytes(rows)) return fail(nullptr, CPMDP_E_WORKSPACE, "MLP workspace too small");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  MlpWs w = carve(ws, rows);
  const FastDiv dm = make_fastdiv(static_cast<uint32_t>(m));
  for (int i = 0; i < n_inst; ++i)
    hipLaunchKernelGGL(features_spread_kernel, dim3(feature_blocks(n)), dim3(256), 0, st, R[i], m, dm,
                       static_cast<float>(gammas[i]), static_cast<float>(slips[i]), S, n,
                       w.X + static_cast<size_t>(i) * n * kXS);
  forward(params, w.X, kXS, rows, w, st, precision == CPMDP_BF16);
  double* part = reinterpret_cast<double*>(w.part);
  for (int i = 0; i < n_inst; ++i)
    hipLaunchKernelGGL(level_partial_kernel, dim3(kLevelBlocks), dim3(256), 0, st,
                       w.y + static_cast<size_t>(i) * n, n, part + i * kLevelBlocks);
  for (int i = 0; i < n_inst; ++i)
    hipLaunchKernelGGL(level_fill_kernel, dim3(std::min(1024, (S + 255) / 256)), dim3(256), 0, st,
                       V0[i], static_cast<int64_t>(S), part + i * kLevelBlocks, kLevelBlocks, n,
                       1.0 / (1.0 - gammas[i]));
  return hipGetLastError() == hipSuccess ? CPMDP_OK
                                         : fail(nullptr, CPMDP_E_DEVICE, "predict_levels launch");
}

int cpmdp_mlp_predict_noalloc(const float* params, const float* R, int32_t m, double gamma,
                              double slip, double* V0, int32_t chunk, int32_t precision,
                              int32_t level, void* stream) {
  if (chunk < 1 || chunk > kStaticRows)
    return mfail("predict_noalloc: chunk must be in [1, 4096] (the static scratch holds the "
                 "workspace of 4096 rows)");
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc) return rc;
  return cpmdp_mlp_predict(params, R, m, gamma, slip, V0, chunk, precision, level, ws,
                           kStaticBytes, stream);
}

}  // extern "C"

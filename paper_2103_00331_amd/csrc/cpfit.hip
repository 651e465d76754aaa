// K11: fitting CP factors to a tabular transition matrix (the decomposition
// step behind the CP form of Sec. 2.2 / Sec. 3, which the paper does not
// specify).  Alternating least squares as in Kolda & Bader, "Tensor
// Decompositions and Applications", SIAM Review 51(3), 2009, Sec. 3.4, on the
// n-way tensor whose mode k pairs the current and next coordinate of dim k:
//     X[u_0, .., u_{n-1}] = P(s' | s),  u_k = i_k m_k + j_k,
// held sparse as the caller's COO triples (s, s', P) in device memory.  A
// rank-R model X ~ sum_r lambda_r a^(0)_r o .. o a^(n-1)_r is the CP form
// P = sum_r lambda_r kron_k T^(k)_r with T^(k)_r = a^(k)_r as an m_k x m_k block.
//
// Per ALS iteration and mode k:
//   M = X_(k) (Khatri-Rao of the other factors)          GPU, over the entries
//   A^(k) = M (Hadamard of the other Gram matrices)^+      host, R x R
//   lambda_r = |A^(k)_r|_2, A^(k)_r /= lambda_r            host
// The matricised-tensor-times-Khatri-Rao product (MTTKRP) is the only step
// that touches the entries: each entry (s, s', p) adds
// p prod_{l != k} A^(l)[u_l, :] to row u_k of M.  Blocks accumulate M in LDS
// (FP64 LDS atomics; M has m_k^2 R <= 8192 words) and store one partial per
// block; a second kernel sums the partials in a fixed order.  The factors
// (sum_k m_k^2 R words, each row padded to an even count so that it is read
// as 16-byte pairs) are read through the caches.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "common.cuh"
#include "handle.h"

#define CP_TRY(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return cpm::fail(nullptr, CPMDP_E_DEVICE,                                    \
                       std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

namespace cpm {

constexpr int kCPMaxRank = 32;
constexpr int kCPMaxLds = 8192;     // m_k^2 R FP64 words of M per block
constexpr int kCPBlocks = 256;      // one block per CU (up to 64 KB of LDS each)
constexpr int kCPThreads = 1024;    // 16 waves per block, 4 per SIMD
constexpr int kCPReduceThreads = 1024;

struct CPArgs {
  const int32_t* rows;
  const int32_t* cols;
  const double* vals;
  int64_t nnz;
  int32_t n, k, R;
  int32_t RP;                       // row stride of A: R rounded up to even
  int32_t m[kMaxDims];
  FastDiv mdiv[kMaxDims];
  int32_t aoff[kMaxDims];           // first row of A^(l) in A (rows of R words)
  const double* A;                  // [sum_l m_l^2][RP], 16-byte aligned
  double* partial;                  // [blocks][m_k^2 R]
};

// Each thread takes runs of 4 consecutive entries (one 16-byte load of the
// states, one of the successors, two of the values: a wave reads 1 KB of
// each array contiguously) and keeps the rows of M it adds to in a few
// register slots (round-robin replacement), so the LDS atomics happen only
// when a row leaves the slots: entries sorted by state reach the same few
// rows of M many times in a row (for the leading dimensions of a grid, a
// whole wave's entries share one or two rows, and per-entry atomics on one
// LDS word serialise).
constexpr int kCPRun = 4;

template <int RMAX, int NT>
__global__ __launch_bounds__(NT) void cp_mttkrp_kernel(CPArgs a) {
  constexpr int kCPSlots = RMAX <= 8 ? 2 : 1;   // registers
  extern __shared__ double Ml[];
  const int len = a.m[a.k] * a.m[a.k] * a.R;
  for (int i = threadIdx.x; i < len; i += NT) Ml[i] = 0.0;
  __syncthreads();
  int key[kCPSlots];
  double acc[kCPSlots][RMAX];
#pragma unroll
  for (int q = 0; q < kCPSlots; ++q) key[q] = -1;
  int victim = 0;
  // one masked set of R atomics for the lanes whose slot vq is taken
  auto flush = [&](int vq) {
    int vkey = -1;
    double vacc[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) vacc[r] = 0.0;
#pragma unroll
    for (int q = 0; q < kCPSlots; ++q)
      if (q == vq) {
        vkey = key[q];
#pragma unroll
        for (int r = 0; r < RMAX; ++r) vacc[r] = acc[q][r];
      }
    if (vkey >= 0) {
#pragma unroll
      for (int r = 0; r < RMAX; ++r)
        if (r < a.R) atomicAdd(&Ml[vkey * a.R + r], vacc[r]);
    }
  };
  const int64_t runs = (a.nnz + kCPRun - 1) / kCPRun;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * NT;
  for (int64_t c = blockIdx.x * NT + threadIdx.x; c < runs; c += stride) {
  const int64_t e0 = c * kCPRun;
  const bool full = e0 + kCPRun <= a.nnz;
  int32_t rs[kCPRun], cs[kCPRun];
  double vs[kCPRun];
  if (full) {
    const int4 r4 = *reinterpret_cast<const int4*>(a.rows + e0);
    const int4 c4 = *reinterpret_cast<const int4*>(a.cols + e0);
    const double2 v0 = *reinterpret_cast<const double2*>(a.vals + e0);
    const double2 v1 = *reinterpret_cast<const double2*>(a.vals + e0 + 2);
    rs[0] = r4.x; rs[1] = r4.y; rs[2] = r4.z; rs[3] = r4.w;
    cs[0] = c4.x; cs[1] = c4.y; cs[2] = c4.z; cs[3] = c4.w;
    vs[0] = v0.x; vs[1] = v0.y; vs[2] = v1.x; vs[3] = v1.y;
  } else {
#pragma unroll
    for (int q = 0; q < kCPRun; ++q) {
      const bool in = e0 + q < a.nnz;
      rs[q] = in ? a.rows[e0 + q] : 0;
      cs[q] = in ? a.cols[e0 + q] : 0;
      vs[q] = in ? a.vals[e0 + q] : 0.0;     // a zero entry adds nothing
    }
  }
#pragma unroll
  for (int q = 0; q < kCPRun; ++q) {
    uint32_t s = static_cast<uint32_t>(rs[q]);
    uint32_t t = static_cast<uint32_t>(cs[q]);
    const double v = vs[q];
    double prod[RMAX];
#pragma unroll
    for (int r = 0; r < RMAX; ++r) prod[r] = v;
    int uk = 0;
    for (int l = a.n - 1; l >= 0; --l) {
      const uint32_t qs = fdiv(s, a.mdiv[l]), qt = fdiv(t, a.mdiv[l]);
      const int i = static_cast<int>(s - qs * a.m[l]), j = static_cast<int>(t - qt * a.m[l]);
      s = qs;
      t = qt;
      const int u = i * a.m[l] + j;
      if (l == a.k) {
        uk = u;
        continue;
      }
      const double2* row =
          reinterpret_cast<const double2*>(a.A + static_cast<size_t>(a.aoff[l] + u) * a.RP);
#pragma unroll
      for (int r = 0; r < RMAX; r += 2)
        if (r < a.R) {
          const double2 f = row[r >> 1];
          prod[r] *= f.x;
          prod[r + 1] *= f.y;   // the padding word when r + 1 == R
        }
    }
    // the slot holding uk, else the victim (flushed first); selects, no
    // per-slot branches, so a wave issues one set of atomics per miss
    int hitq = -1;
#pragma unroll
    for (int q = 0; q < kCPSlots; ++q) hitq = key[q] == uk ? q : hitq;
    if (hitq < 0) {
      flush(victim);
      hitq = victim;
      victim = victim + 1 == kCPSlots ? 0 : victim + 1;
#pragma unroll
      for (int q = 0; q < kCPSlots; ++q)
        if (q == hitq) {
          key[q] = uk;
#pragma unroll
          for (int r = 0; r < RMAX; ++r) acc[q][r] = 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < kCPSlots; ++q)
#pragma unroll
      for (int r = 0; r < RMAX; ++r) acc[q][r] += q == hitq ? prod[r] : 0.0;
  }
  }
#pragma unroll
  for (int q = 0; q < kCPSlots; ++q) flush(q);
  __syncthreads();
  double* dst = a.partial + static_cast<size_t>(blockIdx.x) * len;
  for (int i = threadIdx.x; i < len; i += NT) dst[i] = Ml[i];
}

// out[i] = sum_b partial[b * len + i] in a fixed order: a block covers 64
// consecutive i, its 16 waves take b = w, w + 16, ... (coalesced rows of 64
// words), and the wave sums are added in wave order.
__global__ __launch_bounds__(kCPReduceThreads) void cp_reduce_kernel(const double* partial, int nb,
                                                                     int len, double* out) {
  constexpr int kW = kCPReduceThreads / 64;
  __shared__ double part[kW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  double acc = 0.0;
  if (i < len)
    for (int b = w; b < nb; b += kW) acc += partial[static_cast<size_t>(b) * len + i];
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && i < len) {
    double s = part[0][lane];
    for (int q = 1; q < kW; ++q) s += part[q][lane];
    out[i] = s;
  }
}

// flag bit 0: an entry's state or successor lies outside [0, S) (the MTTKRP
// kernel takes every coordinate in range); bit 1: the entries are not
// strictly increasing in (s, s') (so some pair repeats, which ||X||^2 of the
// reported error does not merge).
__global__ __launch_bounds__(kBlock) void cp_check_kernel(const int32_t* rows, const int32_t* cols,
                                                          int64_t nnz, int32_t S, unsigned* flag) {
  unsigned bad = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t e = blockIdx.x * kBlock + threadIdx.x; e < nnz; e += stride) {
    const int32_t r = rows[e], c = cols[e];
    if (r < 0 || r >= S || c < 0 || c >= S) bad |= 1u;
    if (e + 1 < nnz) {
      const int64_t k0 = static_cast<int64_t>(r) * S + c;
      const int64_t k1 = static_cast<int64_t>(rows[e + 1]) * S + cols[e + 1];
      if (k1 <= k0) bad |= 2u;
    }
  }
  if (bad) atomicOr(flag, bad);
}

// Per-block sums of squares of the entry values (||X||^2 in two passes).
__global__ __launch_bounds__(kBlock) void cp_sumsq_kernel(const double* vals, int64_t nnz,
                                                          double* partial) {
  __shared__ double part[kBlock / 64];
  double acc = 0.0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t e = blockIdx.x * kBlock + threadIdx.x; e < nnz; e += stride) acc += vals[e] * vals[e];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += part[w];
    partial[blockIdx.x] = s;
  }
}

// Moore-Penrose inverse of a symmetric R x R matrix (row-major) by cyclic
// Jacobi rotations: V = Q diag(w) Q^T, V^+ = Q diag(1/w) Q^T over the
// eigenvalues above 1e-15 max |w| (numpy's default cut-off for pinv).
static void sym_pinv(const std::vector<double>& V, int R, std::vector<double>& out) {
  std::vector<double> a(V), q(static_cast<size_t>(R) * R, 0.0);
  for (int i = 0; i < R; ++i) q[i * R + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < R; ++i)
      for (int j = i + 1; j < R; ++j) off += a[i * R + j] * a[i * R + j];
    if (off < 1e-300) break;
    for (int p = 0; p < R; ++p)
      for (int r = p + 1; r < R; ++r) {
        const double apr = a[p * R + r];
        if (std::fabs(apr) < 1e-300) continue;
        const double theta = (a[r * R + r] - a[p * R + p]) / (2.0 * apr);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int i = 0; i < R; ++i) {   // columns p, r
          const double aip = a[i * R + p], air = a[i * R + r];
          a[i * R + p] = c * aip - s * air;
          a[i * R + r] = s * aip + c * air;
        }
        for (int i = 0; i < R; ++i) {   // rows p, r
          const double api = a[p * R + i], ari = a[r * R + i];
          a[p * R + i] = c * api - s * ari;
          a[r * R + i] = s * api + c * ari;
        }
        for (int i = 0; i < R; ++i) {
          const double qip = q[i * R + p], qir = q[i * R + r];
          q[i * R + p] = c * qip - s * qir;
          q[i * R + r] = s * qip + c * qir;
        }
      }
  }
  double wmax = 0.0;
  for (int i = 0; i < R; ++i) wmax = std::max(wmax, std::fabs(a[i * R + i]));
  out.assign(static_cast<size_t>(R) * R, 0.0);
  for (int e = 0; e < R; ++e) {
    const double w = a[e * R + e];
    if (std::fabs(w) <= 1e-15 * wmax || w == 0.0) continue;
    for (int i = 0; i < R; ++i)
      for (int j = 0; j < R; ++j) out[i * R + j] += q[i * R + e] * q[j * R + e] / w;
  }
}

struct CPGeom {
  int n = 0, R = 0;
  int64_t nnz = 0, S = 0;
  std::vector<int32_t> m, aoff;
  int rows_total = 0, len_max = 0, blocks = 1;
};

static int cp_geom(int32_t n_dims, const int64_t* sizes, int64_t nnz, int32_t rank, CPGeom* g) {
  if (!sizes) return fail(nullptr, CPMDP_E_ARG, "sizes is NULL");
  if (n_dims < 1 || n_dims > kMaxDims) return fail(nullptr, CPMDP_E_ARG, "n_dims must be in [1, 8]");
  if (rank < 1 || rank > kCPMaxRank) return fail(nullptr, CPMDP_E_ARG, "rank must be in [1, 32]");
  if (nnz < 1 || nnz >= (int64_t{1} << 31)) return fail(nullptr, CPMDP_E_ARG, "nnz must be in [1, 2^31)");
  g->n = n_dims;
  g->R = rank;
  g->nnz = nnz;
  g->m.assign(sizes, sizes + n_dims);
  g->aoff.resize(n_dims);
  int64_t S = 1, rows = 0;
  g->S = 1;
  int len_max = 0;
  for (int k = 0; k < n_dims; ++k) {
    if (sizes[k] < 1) return fail(nullptr, CPMDP_E_ARG, "sizes must be >= 1");
    S *= sizes[k];
    if (S >= (int64_t{1} << 31)) return fail(nullptr, CPMDP_E_ARG, "state count must be < 2^31");
    const int64_t len = sizes[k] * sizes[k] * rank;
    if (len > kCPMaxLds)
      return fail(nullptr, CPMDP_E_UNSUPPORTED, "m_k^2 * rank must be <= 8192 for every dim");
    g->aoff[k] = static_cast<int32_t>(rows);
    rows += sizes[k] * sizes[k];
    len_max = std::max<int>(len_max, static_cast<int>(len));
  }
  g->S = S;
  g->rows_total = static_cast<int>(rows);
  g->len_max = len_max;
  const int64_t want = (nnz + 4 * kCPThreads - 1) / (4 * kCPThreads);   // >= 4 entries per thread
  g->blocks = static_cast<int>(std::min<int64_t>(std::max<int64_t>(want, 1), kCPBlocks));
  return CPMDP_OK;
}

// Workspace: A [rows][RP], partials [blocks][len_max], M [len_max] (FP64),
// one flag word.
static int cp_row_stride(int R) { return (R + 1) & ~1; }
static size_t cp_ws_bytes(const CPGeom& g) {
  auto al = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
  return al(static_cast<size_t>(g.rows_total) * cp_row_stride(g.R) * 8) +
         al(static_cast<size_t>(g.blocks) * g.len_max * 8) + al(static_cast<size_t>(g.len_max) * 8) +
         256;
}

}  // namespace cpm

using namespace cpm;

extern "C" {

int cpmdp_cp_fit_workspace_bytes(int32_t n_dims, const int64_t* sizes, int64_t nnz, int32_t rank,
                                 size_t* bytes) {
  if (!bytes) return fail(nullptr, CPMDP_E_ARG, "bytes is NULL");
  CPGeom g;
  const int rc = cp_geom(n_dims, sizes, nnz, rank, &g);
  if (rc) return rc;
  *bytes = cp_ws_bytes(g);
  return CPMDP_OK;
}

int cpmdp_cp_fit(int32_t n_dims, const int64_t* sizes, int64_t nnz, const int32_t* rows,
                 const int32_t* cols, const double* vals, int32_t rank, int32_t max_iter, double tol,
                 double* factors, double* lambdas, double* errors, int32_t* iters_out,
                 double* mttkrp_ms, void* workspace, size_t ws_bytes, void* stream) {
  CPGeom g;
  int rc = cp_geom(n_dims, sizes, nnz, rank, &g);
  if (rc) return rc;
  if (!rows || !cols || !vals || !factors || !lambdas)
    return fail(nullptr, CPMDP_E_ARG, "NULL input or output array");
  if (((reinterpret_cast<uintptr_t>(rows) | reinterpret_cast<uintptr_t>(cols) |
        reinterpret_cast<uintptr_t>(vals)) & 15) != 0)
    return fail(nullptr, CPMDP_E_ARG, "rows, cols and vals must be 16-byte aligned");
  if (max_iter < 1) return fail(nullptr, CPMDP_E_ARG, "max_iter must be >= 1");
  if (!(tol >= 0.0)) return fail(nullptr, CPMDP_E_ARG, "tol must be >= 0");
  if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(nullptr, CPMDP_E_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  if (ws_bytes < cp_ws_bytes(g)) return fail(nullptr, CPMDP_E_WORKSPACE, "workspace too small");
  const int n = g.n, R = g.R, RP = cp_row_stride(R);
  int64_t stride = 0;
  for (int k = 0; k < n; ++k) stride += g.m[k] * g.m[k];
  for (int64_t i = 0; i < R * stride; ++i)
    if (!std::isfinite(factors[i])) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite start factor");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(workspace);
  auto al = [](size_t x) { return (x + 255) & ~static_cast<size_t>(255); };
  double* dA = reinterpret_cast<double*>(base);
  double* dP = reinterpret_cast<double*>(base + al(static_cast<size_t>(g.rows_total) * RP * 8));
  double* dM = reinterpret_cast<double*>(base + al(static_cast<size_t>(g.rows_total) * RP * 8) +
                                         al(static_cast<size_t>(g.blocks) * g.len_max * 8));
  unsigned* dflag = reinterpret_cast<unsigned*>(reinterpret_cast<char*>(dM) +
                                                al(static_cast<size_t>(g.len_max) * 8));
  // host factors, mode-major [rows][R]
  std::vector<std::vector<double>> A(n);
  for (int k = 0; k < n; ++k) {
    const int rk = g.m[k] * g.m[k];
    A[k].resize(static_cast<size_t>(rk) * R);
    for (int r = 0; r < R; ++r)
      for (int u = 0; u < rk; ++u) A[k][u * R + r] = factors[r * stride + (g.aoff[k]) + u];
  }
  // device copy with rows padded to RP words (the padding stays zero)
  std::vector<double> flatA(static_cast<size_t>(g.rows_total) * RP, 0.0);
  auto pad_rows = [&](int k, double* dst) {
    const int rk = g.m[k] * g.m[k];
    for (int u = 0; u < rk; ++u)
      for (int r = 0; r < R; ++r) dst[static_cast<size_t>(u) * RP + r] = A[k][u * R + r];
  };
  for (int k = 0; k < n; ++k) pad_rows(k, flatA.data() + static_cast<size_t>(g.aoff[k]) * RP);
  CP_TRY(hipMemcpyAsync(dA, flatA.data(), flatA.size() * 8, hipMemcpyHostToDevice, st));
  auto gram = [&](int k) {
    const int rk = g.m[k] * g.m[k];
    std::vector<double> G(static_cast<size_t>(R) * R, 0.0);
    for (int u = 0; u < rk; ++u)
      for (int p = 0; p < R; ++p)
        for (int q = 0; q < R; ++q) G[p * R + q] += A[k][u * R + p] * A[k][u * R + q];
    return G;
  };
  std::vector<std::vector<double>> G(n);
  for (int k = 0; k < n; ++k) G[k] = gram(k);
  // coordinates in range, and ||X||^2
  launch_fill_u32(dflag, 1, 0u, st);
  hipLaunchKernelGGL(cp_check_kernel, dim3(g.blocks), dim3(kBlock), 0, st, rows, cols, g.nnz,
                     static_cast<int32_t>(g.S), dflag);
  hipLaunchKernelGGL(cp_sumsq_kernel, dim3(g.blocks), dim3(kBlock), 0, st, vals, g.nnz, dP);
  hipLaunchKernelGGL(cp_reduce_kernel, dim3(1), dim3(kCPReduceThreads), 0, st, dP, g.blocks, 1, dM);
  double normX2 = 0.0;
  unsigned flag = 0;
  CP_TRY(hipMemcpyAsync(&normX2, dM, 8, hipMemcpyDeviceToHost, st));
  CP_TRY(hipMemcpyAsync(&flag, dflag, 4, hipMemcpyDeviceToHost, st));
  CP_TRY(hipStreamSynchronize(st));
  CP_TRY(hipGetLastError());
  if (flag & 1u) return fail(nullptr, CPMDP_E_ARG, "an entry's state or successor is outside [0, S)");
  if (flag & 2u)
    return fail(nullptr, CPMDP_E_ARG, "entries must be distinct and sorted by (state, successor)");
  if (!std::isfinite(normX2)) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite entry value");
  if (normX2 <= 0.0) return fail(nullptr, CPMDP_E_ARG, "all entry values are zero");
  CPArgs a{};
  a.rows = rows;
  a.cols = cols;
  a.vals = vals;
  a.nnz = g.nnz;
  a.n = n;
  a.R = R;
  a.RP = RP;
  for (int k = 0; k < n; ++k) {
    a.m[k] = g.m[k];
    a.mdiv[k] = make_fastdiv(static_cast<uint32_t>(g.m[k]));
    a.aoff[k] = g.aoff[k];
  }
  a.A = dA;
  a.partial = dP;
  struct Events {     // destroyed on every return path
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } evs;
  if (mttkrp_ms) {
    CP_TRY(hipEventCreate(&evs.e0));
    CP_TRY(hipEventCreate(&evs.e1));
  }
  hipEvent_t ev0 = evs.e0, ev1 = evs.e1;
  double t_ms = 0.0;
  int64_t t_n = 0;
  std::vector<double> lam(R, 1.0), M, Vp, Vinv;
  double prev = INFINITY;
  int it = 0;
  int out_rc = CPMDP_OK;
  for (it = 0; it < max_iter; ++it) {
    for (int k = 0; k < n; ++k) {
      const int rk = g.m[k] * g.m[k], len = rk * R;
      a.k = k;
      const size_t sh = static_cast<size_t>(len) * 8;
      const LaunchTiming t0{ev0, nullptr}, t1{nullptr, ev1};
      const LaunchTiming* tm0 = mttkrp_ms ? &t0 : nullptr;
      if (R <= 8) klaunch(cp_mttkrp_kernel<8, kCPThreads>, dim3(g.blocks), dim3(kCPThreads), sh, st, tm0, a);
      else if (R <= 16) klaunch(cp_mttkrp_kernel<16, kCPThreads>, dim3(g.blocks), dim3(kCPThreads), sh, st, tm0, a);
      else klaunch(cp_mttkrp_kernel<32, kCPThreads / 2>, dim3(g.blocks), dim3(kCPThreads / 2), sh, st, tm0, a);
      klaunch(cp_reduce_kernel, dim3((len + 63) / 64), dim3(kCPReduceThreads), 0, st,
              mttkrp_ms ? &t1 : nullptr, static_cast<const double*>(dP), g.blocks, len, dM);
      M.assign(static_cast<size_t>(len), 0.0);
      CP_TRY(hipMemcpyAsync(M.data(), dM, static_cast<size_t>(len) * 8,
                                      hipMemcpyDeviceToHost, st));
      CP_TRY(hipStreamSynchronize(st));
      CP_TRY(hipGetLastError());
      if (mttkrp_ms) {
        float ms = 0.f;
        CP_TRY(hipEventElapsedTime(&ms, ev0, ev1));
        t_ms += ms;
        ++t_n;
      }
      // A^(k) = M V^+, V = Hadamard product of the other Gram matrices
      Vp.assign(static_cast<size_t>(R) * R, 1.0);
      for (int l = 0; l < n; ++l)
        if (l != k)
          for (int i = 0; i < R * R; ++i) Vp[i] *= G[l][i];
      sym_pinv(Vp, R, Vinv);
      for (int u = 0; u < rk; ++u)
        for (int r = 0; r < R; ++r) {
          double acc = 0.0;
          for (int q = 0; q < R; ++q) acc += M[u * R + q] * Vinv[q * R + r];
          A[k][u * R + r] = acc;
        }
      for (int r = 0; r < R; ++r) {
        double s2 = 0.0;
        for (int u = 0; u < rk; ++u) s2 += A[k][u * R + r] * A[k][u * R + r];
        lam[r] = std::sqrt(s2);
        if (lam[r] > 0.0)
          for (int u = 0; u < rk; ++u) A[k][u * R + r] /= lam[r];
      }
      G[k] = gram(k);
      double* hk = flatA.data() + static_cast<size_t>(g.aoff[k]) * RP;
      pad_rows(k, hk);
      CP_TRY(hipMemcpyAsync(dA + static_cast<size_t>(g.aoff[k]) * RP, hk,
                            static_cast<size_t>(rk) * RP * 8, hipMemcpyHostToDevice, st));
    }
    // relative error from ||X||^2, <X, X_hat> (the last mode's M against its
    // new factor) and ||X_hat||^2 = lambda^T (Hadamard of all Grams) lambda
    const int kl = n - 1, rl = g.m[kl] * g.m[kl];
    double inner = 0.0, nh = 0.0;
    for (int r = 0; r < R; ++r) {
      double s = 0.0;
      for (int u = 0; u < rl; ++u) s += M[u * R + r] * A[kl][u * R + r];
      inner += lam[r] * s;
    }
    for (int p = 0; p < R; ++p)
      for (int q = 0; q < R; ++q) {
        double h = lam[p] * lam[q];
        for (int l = 0; l < n; ++l) h *= G[l][p * R + q];
        nh += h;
      }
    const double err = std::sqrt(std::max(0.0, normX2 - 2.0 * inner + nh)) / std::sqrt(normX2);
    if (!std::isfinite(err)) {
      out_rc = fail(nullptr, CPMDP_E_NONFINITE, "non-finite fit");
      break;
    }
    if (errors) errors[it] = err;
    if (std::fabs(prev - err) <= tol) {
      ++it;
      break;
    }
    prev = err;
  }
  // the factor uploads read flatA, which ends with this call
  const hipError_t se = hipStreamSynchronize(st);
  if (out_rc) return out_rc;
  if (se != hipSuccess)
    return fail(nullptr, CPMDP_E_DEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(se));
  for (int k = 0; k < n; ++k) {
    const int rk = g.m[k] * g.m[k];
    for (int r = 0; r < R; ++r)
      for (int u = 0; u < rk; ++u) factors[r * stride + g.aoff[k] + u] = A[k][u * R + r];
  }
  for (int r = 0; r < R; ++r) lambdas[r] = lam[r];
  if (iters_out) *iters_out = it;
  if (mttkrp_ms) *mttkrp_ms = t_n ? t_ms / t_n : 0.0;
  return CPMDP_OK;
}

}  // extern "C"

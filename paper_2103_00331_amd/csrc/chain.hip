// K2: Bellman backup for general (dense) factors, as chains of mode products.
//
// A rank term applies kron_k T^{(k)} to V, i.e. the mode-k product of the
// n-way value tensor with every factor, (V x_k T)[..i..] = sum_j T[i,j] V[..j..]
// (the CP form of Sec. 2.2 applied without ever forming P_a).  Mode products
// along different modes commute, so the dims are split into a row group
// [0, n1) and a column group [n1, n) and every term is applied in two passes:
//
//   pass 1 (one block per row r): the slab V[r, :] (all column dims) sits in
//     LDS; for each term its column-group mode products run in place in LDS
//     and the result is written to the intermediate W_t, in the tiled layout
//     [tile][r][c_lo] (c = tile * CT + c_lo) so that pass 2 reads one
//     contiguous block per tile.
//   pass 2 (one block per tile of CT columns): for each action and each of
//     its terms, the tile W_t[tile] (all rows x CT columns) is loaded into
//     LDS, the row-group mode products run in place, and lambda * result is
//     accumulated per state in registers; then the Q-value of Eq. 1, the
//     max / argmax over actions, V' and the sup-norm residual are fused.
//
// Identity factors are skipped.  An in-place mode product lets each thread
// hold whole fibers in registers: load fiber, barrier, write the m outputs.
// LDS indices are padded by one word per 32 to break bank conflicts of
// strided fibers.
#include <type_traits>

#include "common.cuh"

namespace cpm {

__device__ __forceinline__ int lpad(int i) { return i + (i >> 5); }

// In-place mode product on an LDS array viewed as [outer][m][inner]:
// X[o, i, in] <- sum_j Tk[i, j] X[o, j, in].
template <typename T, int MMAX>
__device__ __forceinline__ void mode_product_lds(T* X, int outer, int m, int inner,
                                                 const T* __restrict__ Tk) {
  const int F = outer * inner;
  for (int f0 = 0; f0 < F; f0 += blockDim.x) {
    const int f = f0 + threadIdx.x;
    const bool act = f < F;
    T x[MMAX];
    int base = 0;
    if (act) {
      const int o = f / inner;
      const int in = f - o * inner;
      base = o * m * inner + in;
#pragma unroll
      for (int j = 0; j < MMAX; ++j)
        if (j < m) x[j] = X[lpad(base + j * inner)];
    }
    __syncthreads();
    if (act) {
      for (int i = 0; i < m; ++i) {
        const T* Ti = Tk + i * m;
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < MMAX; ++j)
          if (j < m) acc = fma(Ti[j], x[j], acc);
        X[lpad(base + i * inner)] = acc;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------ MFMA path
// For m_k <= 16 a mode product is a batch of 16 x 16 matrix-vector products
// T (16 x 16, zero-padded) times 16-element fibers: one 16 x 16 x 16 matrix
// product per block of 16 fibers.  Matrix-core layout (wave of 64 lanes,
// lane l: column c = l % 16, group g = l / 16):
//   fp32 16x16x4 : A[i = c][k = 4q + g], B[k = 4q + g][fiber c], q = 0..3
//   bf16 16x16x16: A[i = c][k = 4g + r], B[k = 4g + r][fiber c], r = 0..3
//   result       : D[i = 4g + r][fiber c], r = 0..3 (FP32 accumulation)
// The BF16 unit splits factor and fiber values into hi + lo BF16 parts
// (x_hi = bf16(x), x_lo = bf16(x - x_hi)) and accumulates lo*hi, hi*lo,
// hi*hi; the dropped lo*lo term and the lo rounding leave a relative error
// of a few 2^-16 per mode product instead of 2^-8.
// A wave owns whole blocks: it reads all 16 x 16 inputs of a block before its
// matrix products and writes the outputs to the same LDS slots afterwards, so
// the product is in place without a barrier between blocks.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

enum { MM_VALU = 0, MM_F32 = 1, MM_BF16 = 2 };

__device__ __forceinline__ uint32_t bf16_bits(float x) {   // round to nearest even
  const uint32_t u = __float_as_uint(x);
  return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

template <int MM>
__device__ __forceinline__ void mode_product_mfma(float* X, int outer, int m, int inner,
                                                  const float* __restrict__ Tk,
                                                  const uint16_t* __restrict__ Th,
                                                  const uint16_t* __restrict__ Tl) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int F = outer * inner;
  const int nblk = (F + 15) >> 4;
  float a32[4];
  s4v ahi, alo;
  if (MM == MM_F32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = 4 * q + g;
      a32[q] = (c < m && k < m) ? Tk[c * m + k] : 0.f;
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int k = 4 * g + r;
      const bool in = c < m && k < m;
      ahi[r] = in ? static_cast<short>(Th[c * m + k]) : static_cast<short>(0);
      alo[r] = in ? static_cast<short>(Tl[c * m + k]) : static_cast<short>(0);
    }
  }
  for (int b = wave; b < nblk; b += nw) {
    const int f = b * 16 + c;
    const bool ok = f < F;
    int base = 0;
    if (ok) {
      const int o = f / inner;
      base = o * m * inner + (f - o * inner);
    }
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    if (MM == MM_F32) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = 4 * q + g;
        const float bv = (ok && k < m) ? X[lpad(base + k * inner)] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a32[q], bv, acc, 0, 0, 0);
      }
    } else {
      s4v bhi, blo;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 4 * g + r;
        const float x = (ok && k < m) ? X[lpad(base + k * inner)] : 0.f;
        const uint32_t h = bf16_bits(x);
        bhi[r] = static_cast<short>(h);
        blo[r] = static_cast<short>(bf16_bits(x - bf16_value(h)));
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 4 * g + r;
      if (ok && i < m) X[lpad(base + i * inner)] = acc[r];
    }
  }
  __syncthreads();
}

// Mode product of one term's factor along one mode, on the chosen unit.
template <typename T, int MMAX, int MM>
__device__ __forceinline__ void mode_product(T* X, int outer, int m, int inner, const T* Tk,
                                             const uint16_t* Th, const uint16_t* Tl) {
  if constexpr (MM == MM_VALU) {
    mode_product_lds<T, MMAX>(X, outer, m, inner, Tk);
  } else {
    mode_product_mfma<MM>(X, outer, m, inner, Tk, Th, Tl);
  }
}

constexpr int kPass1Block = 256;
constexpr int kPass2Block = 512;

template <typename T, int MMAX, int MM>
__global__ __launch_bounds__(kPass1Block) void chain_pass1(ChainArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  const int C = a.g.C;
  T* vs = reinterpret_cast<T*>(smem_raw);
  T* ws = vs + lpad(C) + 1;
  const int r = xcd_block(blockIdx.x, gridDim.x);
  const T* Vrow = a.V + static_cast<int64_t>(r) * C;
  const T cs = a.shift_keys ? static_cast<T>(midrange(a.shift_keys)) : T(0);
  for (int c = threadIdx.x; c < C; c += blockDim.x) vs[lpad(c)] = Vrow[c] - cs;
  __syncthreads();
  const int n = a.g.n;
  for (int t = 0; t < a.nterms; ++t) {
    for (int c = threadIdx.x; c < C; c += blockDim.x) ws[lpad(c)] = vs[lpad(c)];
    __syncthreads();
    int outer = 1, inner = C;
    for (int k = a.g.n1; k < n; ++k) {
      const int m = a.g.size[k];
      inner /= m;
      if (a.kinds[t * n + k] != F_IDENT) {
        const int64_t fo = static_cast<int64_t>(t) * a.g.term_stride + a.g.fac_off[k];
        mode_product<T, MMAX, MM>(ws, outer, m, inner, a.fac + fo, a.facbf + fo, a.facbf_lo + fo);
      }
      outer *= m;
    }
    T* Wt = a.W + static_cast<int64_t>(t) * a.g.w_term_stride;
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
      const int tile = c >> a.g.ct_shift, clo = c & (a.g.CT - 1);
      Wt[(static_cast<int64_t>(tile) * a.g.Rr + r) * a.g.CT + clo] = ws[lpad(c)];
    }
    __syncthreads();
  }
}

template <typename T, int MMAX, int MODE, int EPT, int MM>
__global__ __launch_bounds__(kPass2Block) void chain_pass2(ChainArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);
  __shared__ int act_used[kMaxActions + 1];
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int CT = a.g.CT, C = a.g.C, n1 = a.g.n1, n = a.g.n;
  const int TE = a.g.Rr * CT;

  T acc[EPT], best[EPT], qold[EPT];
  int bi[EPT], pold[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    acc[j] = T(0);
    best[j] = -INFINITY;
    qold[j] = -INFINITY;
    bi[j] = 0;
    pold[j] = -1;
  }
  auto state_of = [&](int e, bool& valid) -> int {
    const int r = e >> a.g.ct_shift, clo = e & (CT - 1);
    const int c = tile * CT + clo;
    valid = (e < TE) && (c < C);
    return r * C + c;
  };

  T tol = T(0);
  if (MODE == MODE_GREEDY) tol = static_cast<T>(tie_tol(a.vmax_bits));
  // shift c: pass 1 (or, with a single pass, the load below) works on V - c
  const T cs = a.shift_keys ? static_cast<T>(midrange(a.shift_keys)) : T(0);
  const T cs_in = (n1 == n) ? cs : T(0);
  const bool need_pi = (MODE == MODE_EVAL || MODE == MODE_RESID) ||
                       (MODE == MODE_GREEDY && a.pi_in != nullptr);
  if (MODE == MODE_EVAL || MODE == MODE_RESID) {
    for (int i = threadIdx.x; i < a.A; i += blockDim.x) act_used[i] = 0;
    __syncthreads();
  }
  if (need_pi) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      bool v;
      const int s = state_of(threadIdx.x + j * kPass2Block, v);
      if (v) {
        pold[j] = a.pi_in[s];
        if (MODE == MODE_EVAL || MODE == MODE_RESID) act_used[pold[j]] = 1;
      }
    }
  }
  if (MODE == MODE_EVAL || MODE == MODE_RESID) __syncthreads();

  const int64_t tile_off = static_cast<int64_t>(tile) * TE;
  for (int act = 0; act < a.A; ++act) {
    if ((MODE == MODE_EVAL || MODE == MODE_RESID) && !act_used[act]) continue;
    if (MODE == MODE_MAX || MODE == MODE_GREEDY) {
#pragma unroll
      for (int j = 0; j < EPT; ++j) acc[j] = T(0);
    }
    for (int t = a.term_start[act]; t < a.term_start[act + 1]; ++t) {
      const T* Wt = a.W + static_cast<int64_t>(t) * a.g.w_term_stride + tile_off;
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = threadIdx.x + j * kPass2Block;
        if (e < TE) X[lpad(e)] = Wt[e] - cs_in;
      }
      __syncthreads();
      int outer = 1, inner = TE;
      for (int k = 0; k < n1; ++k) {
        const int m = a.g.size[k];
        inner /= m;
        if (a.kinds[t * n + k] != F_IDENT) {
          const int64_t fo = static_cast<int64_t>(t) * a.g.term_stride + a.g.fac_off[k];
          mode_product<T, MMAX, MM>(X, outer, m, inner, a.fac + fo, a.facbf + fo, a.facbf_lo + fo);
        }
        outer *= m;
      }
      const T lam = a.lam[t];
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = threadIdx.x + j * kPass2Block;
        if (e < TE) {
          const T x = X[lpad(e)];
          if (MODE == MODE_EVAL || MODE == MODE_RESID) {
            if (pold[j] == act) acc[j] = fma(lam, x, acc[j]);
          } else {
            acc[j] = fma(lam, x, acc[j]);
          }
        }
      }
      __syncthreads();
    }
    if (MODE == MODE_MAX) {
#pragma unroll
      for (int j = 0; j < EPT; ++j) best[j] = acc[j] > best[j] ? acc[j] : best[j];
    } else if (MODE == MODE_GREEDY) {
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        bool v;
        const int s = state_of(threadIdx.x + j * kPass2Block, v);
        if (v) {
          const T g = is_terminal(a.term_bits, s) ? T(0) : a.gamma;
          const T q = fma(g, acc[j] + cs, a.R[s]);
          tie_update(q, act, tol, best[j], bi[j]);
          if (act == pold[j]) qold[j] = q;
        }
      }
    }
  }

  double res = 0.0;
  unsigned changed = 0;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    bool v;
    const int s = state_of(threadIdx.x + j * kPass2Block, v);
    if (!v) continue;
    const T c = a.V[s];
    if (MODE == MODE_GREEDY) {
      int pnew = bi[j];
      if (pold[j] >= 0 && qold[j] >= best[j] - tol) pnew = pold[j];
      changed += (pold[j] >= 0 && pnew != pold[j]) ? 1u : 0u;
      if (a.pi_out) a.pi_out[s] = pnew;
      if (a.Vout) a.Vout[s] = best[j];
      res = nanmax(res, fabs(static_cast<double>(best[j]) - static_cast<double>(c)));
    } else {
      const T g = is_terminal(a.term_bits, s) ? T(0) : a.gamma;
      const T vnew = fma(g, (MODE == MODE_MAX ? best[j] : acc[j]) + cs, a.R[s]);
      const double d = static_cast<double>(vnew) - static_cast<double>(c);
      if (MODE == MODE_RESID) {
        a.r_out[s] = static_cast<float>(d);
      } else {
        a.Vout[s] = vnew;
      }
      res = nanmax(res, fabs(d));
    }
  }
  block_max_to_slot(res, a.res_slot);
  if (MODE == MODE_GREEDY && a.change_count) block_sum_to_counter(changed, a.change_count);
}

// --------------------------------------------------------------- launchers

static int pick_mmax(int m) {
  if (m <= 4) return 4;
  if (m <= 16) return 16;
  return 32;
}

template <typename T, int MMAX, int MM>
static void launch_pass1_m(const ChainArgs<T>& a, hipStream_t st) {
  const size_t sh = sizeof(T) * (2 * (static_cast<size_t>(a.g.C) + (a.g.C >> 5) + 1) + 2);
  hipLaunchKernelGGL((chain_pass1<T, MMAX, MM>), dim3(a.g.Rr), dim3(kPass1Block), sh, st, a);
}

template <typename T, int MMAX, int MODE, int MM>
static void launch_pass2_mm(const ChainArgs<T>& a, hipStream_t st) {
  const int TE = a.g.Rr * a.g.CT;
  const int ept = (TE + kPass2Block - 1) / kPass2Block;
  const size_t sh = sizeof(T) * (static_cast<size_t>(TE) + (TE >> 5) + 1);
  const dim3 grid(a.g.ntiles), block(kPass2Block);
  if (ept <= 2) hipLaunchKernelGGL((chain_pass2<T, MMAX, MODE, 2, MM>), grid, block, sh, st, a);
  else if (ept <= 8) hipLaunchKernelGGL((chain_pass2<T, MMAX, MODE, 8, MM>), grid, block, sh, st, a);
  else if (ept <= 16) hipLaunchKernelGGL((chain_pass2<T, MMAX, MODE, 16, MM>), grid, block, sh, st, a);
  else hipLaunchKernelGGL((chain_pass2<T, MMAX, MODE, 32, MM>), grid, block, sh, st, a);
}

template <typename T, int MMAX, int MM>
static void launch_pass2_m(const ChainArgs<T>& a, int mode, hipStream_t st) {
  switch (mode) {
    case MODE_MAX: launch_pass2_mm<T, MMAX, MODE_MAX, MM>(a, st); break;
    case MODE_GREEDY: launch_pass2_mm<T, MMAX, MODE_GREEDY, MM>(a, st); break;
    case MODE_EVAL: launch_pass2_mm<T, MMAX, MODE_EVAL, MM>(a, st); break;
    default: launch_pass2_mm<T, MMAX, MODE_RESID, MM>(a, st); break;
  }
}

// Unit of one group's mode products: matrix cores when every mode of the
// group has m_k <= 16 (FP32 from 5 up, BF16 always), vector ALUs otherwise.
static int pick_unit(int mmax, int unit) {
  if (unit == CHAIN_BF16) return mmax <= 16 ? MM_BF16 : MM_VALU;
  if (unit == CHAIN_F32_MFMA) return (mmax > 4 && mmax <= 16) ? MM_F32 : MM_VALU;
  return MM_VALU;
}

template <typename T>
static void launch_pass1(const ChainArgs<T>& a, int mm, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (mm == MM_F32) return launch_pass1_m<T, 16, MM_F32>(a, st);
    if (mm == MM_BF16) return launch_pass1_m<T, 16, MM_BF16>(a, st);
  }
  switch (pick_mmax(a.g.mmax_col)) {
    case 4: return launch_pass1_m<T, 4, MM_VALU>(a, st);
    case 16: return launch_pass1_m<T, 16, MM_VALU>(a, st);
    default: return launch_pass1_m<T, 32, MM_VALU>(a, st);
  }
}

template <typename T>
static void launch_pass2(const ChainArgs<T>& a, int mode, int mm, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    if (mm == MM_F32) return launch_pass2_m<T, 16, MM_F32>(a, mode, st);
    if (mm == MM_BF16) return launch_pass2_m<T, 16, MM_BF16>(a, mode, st);
  }
  switch (pick_mmax(a.g.mmax_row)) {
    case 4: return launch_pass2_m<T, 4, MM_VALU>(a, mode, st);
    case 16: return launch_pass2_m<T, 16, MM_VALU>(a, mode, st);
    default: return launch_pass2_m<T, 32, MM_VALU>(a, mode, st);
  }
}

template <typename T>
void launch_chain(const ChainArgs<T>& a, int mode, int unit, hipStream_t st) {
  const bool f32 = std::is_same<T, float>::value;
  if (a.g.n1 < a.g.n) launch_pass1(a, f32 ? pick_unit(a.g.mmax_col, unit) : MM_VALU, st);
  launch_pass2(a, mode, f32 ? pick_unit(a.g.mmax_row, unit) : MM_VALU, st);
}

template void launch_chain<double>(const ChainArgs<double>&, int, int, hipStream_t);
template void launch_chain<float>(const ChainArgs<float>&, int, int, hipStream_t);

}  // namespace cpm

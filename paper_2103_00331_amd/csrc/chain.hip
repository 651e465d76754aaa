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

constexpr int kPass1Block = 256;
constexpr int kPass2Block = 512;

template <typename T, int MMAX>
__global__ __launch_bounds__(kPass1Block) void chain_pass1(ChainArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  const int C = a.g.C;
  T* vs = reinterpret_cast<T*>(smem_raw);
  T* ws = vs + lpad(C) + 1;
  const int r = xcd_block(blockIdx.x, gridDim.x);
  const T* Vrow = a.V + static_cast<int64_t>(r) * C;
  for (int c = threadIdx.x; c < C; c += blockDim.x) vs[lpad(c)] = Vrow[c];
  __syncthreads();
  const int n = a.g.n;
  for (int t = 0; t < a.nterms; ++t) {
    for (int c = threadIdx.x; c < C; c += blockDim.x) ws[lpad(c)] = vs[lpad(c)];
    __syncthreads();
    int outer = 1, inner = C;
    for (int k = a.g.n1; k < n; ++k) {
      const int m = a.g.size[k];
      inner /= m;
      if (a.kinds[t * n + k] != F_IDENT)
        mode_product_lds<T, MMAX>(ws, outer, m, inner,
                                  a.fac + static_cast<int64_t>(t) * a.g.term_stride + a.g.fac_off[k]);
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

template <typename T, int MMAX, int MODE, int EPT>
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
        if (e < TE) X[lpad(e)] = Wt[e];
      }
      __syncthreads();
      int outer = 1, inner = TE;
      for (int k = 0; k < n1; ++k) {
        const int m = a.g.size[k];
        inner /= m;
        if (a.kinds[t * n + k] != F_IDENT)
          mode_product_lds<T, MMAX>(X, outer, m, inner,
                                    a.fac + static_cast<int64_t>(t) * a.g.term_stride + a.g.fac_off[k]);
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
          const T q = fma(g, acc[j], a.R[s]);
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
      const T vnew = fma(g, MODE == MODE_MAX ? best[j] : acc[j], a.R[s]);
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

template <typename T, int MMAX>
static void launch_pass1_m(const ChainArgs<T>& a, hipStream_t st) {
  const size_t sh = sizeof(T) * (2 * (static_cast<size_t>(a.g.C) + (a.g.C >> 5) + 1) + 2);
  hipLaunchKernelGGL((chain_pass1<T, MMAX>), dim3(a.g.Rr), dim3(kPass1Block), sh, st, a);
}

template <typename T, int MMAX, int MODE>
static void launch_pass2_mm(const ChainArgs<T>& a, hipStream_t st) {
  const int TE = a.g.Rr * a.g.CT;
  const int ept = (TE + kPass2Block - 1) / kPass2Block;
  const size_t sh = sizeof(T) * (static_cast<size_t>(TE) + (TE >> 5) + 1);
  const dim3 grid(a.g.ntiles), block(kPass2Block);
  if (ept <= 2) hipLaunchKernelGGL((chain_pass2<T, MMAX, MODE, 2>), grid, block, sh, st, a);
  else if (ept <= 8) hipLaunchKernelGGL((chain_pass2<T, MMAX, MODE, 8>), grid, block, sh, st, a);
  else if (ept <= 16) hipLaunchKernelGGL((chain_pass2<T, MMAX, MODE, 16>), grid, block, sh, st, a);
  else hipLaunchKernelGGL((chain_pass2<T, MMAX, MODE, 32>), grid, block, sh, st, a);
}

template <typename T, int MMAX>
static void launch_pass2_m(const ChainArgs<T>& a, int mode, hipStream_t st) {
  switch (mode) {
    case MODE_MAX: launch_pass2_mm<T, MMAX, MODE_MAX>(a, st); break;
    case MODE_GREEDY: launch_pass2_mm<T, MMAX, MODE_GREEDY>(a, st); break;
    case MODE_EVAL: launch_pass2_mm<T, MMAX, MODE_EVAL>(a, st); break;
    default: launch_pass2_mm<T, MMAX, MODE_RESID>(a, st); break;
  }
}

template <typename T>
void launch_chain(const ChainArgs<T>& a, int mode, hipStream_t st) {
  if (a.g.n1 < a.g.n) {
    switch (pick_mmax(a.g.mmax_col)) {
      case 4: launch_pass1_m<T, 4>(a, st); break;
      case 16: launch_pass1_m<T, 16>(a, st); break;
      default: launch_pass1_m<T, 32>(a, st); break;
    }
  }
  switch (pick_mmax(a.g.mmax_row)) {
    case 4: launch_pass2_m<T, 4>(a, mode, st); break;
    case 16: launch_pass2_m<T, 16>(a, mode, st); break;
    default: launch_pass2_m<T, 32>(a, mode, st); break;
  }
}

template void launch_chain<double>(const ChainArgs<double>&, int, hipStream_t);
template void launch_chain<float>(const ChainArgs<float>&, int, hipStream_t);

}  // namespace cpm

// K1: Bellman backup for factors that are identities or clamped +-1 shifts.
//
// With every rank term of the form I (x) ... (x) shift (x) ... (x) I, the mode
// products of V with the factors reduce to reading V at the state itself or
// at one axis neighbour (clamped at the grid edge: a move off the grid stays
// put).  Terms of one action that read the same neighbour are summed into one
// weight, so an action is a (2n+1)-point weighted stencil:
//     (P_a V)(s) = sum_p w[a][p] V(nbr_p(s)),   w[a][p] = sum of lambda_{a,r}
// over the terms whose shift is point p.  One thread owns one state: it reads
// V at its 2n+1 points (the neighbours mostly hit L2), R(s) and the terminal
// bit, evaluates every action, and fuses the max / argmax (Eq. 1), the write
// of V' and a block-reduced sup-norm residual.  The sweep streams
// V, R and V' once: 3 words per state.
#include "common.cuh"

namespace cpm {

template <typename T, int N, int MODE>
__global__ __launch_bounds__(kBlock) void stencil_kernel(StencilArgs<T> a) {
  constexpr int P = 2 * N + 1;
  extern __shared__ unsigned char smem_raw[];
  T* wsh = reinterpret_cast<T*>(smem_raw);
  if (MODE == MODE_EVAL || MODE == MODE_RESID) {
    const int nw = a.A * P;
    for (int i = threadIdx.x; i < nw; i += blockDim.x) wsh[i] = a.w[i];
    __syncthreads();
  }
  const int blk = xcd_block(blockIdx.x, a.nblocks);
  const int s = blk * kBlock + threadIdx.x;
  double res = 0.0;
  unsigned changed = 0;
  if (s < a.g.S) {
    int idx[N];
    uint32_t rem = static_cast<uint32_t>(s);
#pragma unroll
    for (int k = N - 1; k > 0; --k) {
      const uint32_t q = fdiv(rem, a.g.div[k]);
      idx[k] = static_cast<int>(rem - q * static_cast<uint32_t>(a.g.size[k]));
      rem = q;
    }
    idx[0] = static_cast<int>(rem);

    T nb[P];
    const T c = a.V[s];
    nb[0] = c;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int st = a.g.stride[k];
      nb[1 + 2 * k] = (idx[k] < a.g.size[k] - 1) ? a.V[s + st] : c;
      nb[2 + 2 * k] = (idx[k] > 0) ? a.V[s - st] : c;
    }
    const T g = is_terminal(a.term_bits, s) ? T(0) : a.gamma;
    const T rs = a.R[s];

    if (MODE == MODE_MAX) {
      T best = -INFINITY;
      for (int act = 0; act < a.A; ++act) {
        const T* wa = a.w + act * P;
        T acc = T(0);
#pragma unroll
        for (int p = 0; p < P; ++p) acc = fma(wa[p], nb[p], acc);
        best = acc > best ? acc : best;
      }
      const T v = fma(g, best, rs);
      a.Vout[s] = v;
      res = fabs(static_cast<double>(v) - static_cast<double>(c));
    } else if (MODE == MODE_GREEDY) {
      const T tol = static_cast<T>(tie_tol(a.vmax_bits));
      const int pold = a.pi_in ? a.pi_in[s] : -1;
      T best = -INFINITY, qold = -INFINITY;
      int bi = 0;
      for (int act = 0; act < a.A; ++act) {
        const T* wa = a.w + act * P;
        T acc = T(0);
#pragma unroll
        for (int p = 0; p < P; ++p) acc = fma(wa[p], nb[p], acc);
        const T q = fma(g, acc, rs);
        tie_update(q, act, tol, best, bi);
        if (act == pold) qold = q;
      }
      int pnew = bi;
      if (pold >= 0 && qold >= best - tol) pnew = pold;
      changed = (pold >= 0 && pnew != pold) ? 1u : 0u;
      if (a.pi_out) a.pi_out[s] = pnew;
      if (a.Vout) a.Vout[s] = best;
      res = fabs(static_cast<double>(best) - static_cast<double>(c));
    } else {
      const T* wa = wsh + a.pi_in[s] * P;
      T acc = T(0);
#pragma unroll
      for (int p = 0; p < P; ++p) acc = fma(wa[p], nb[p], acc);
      const T v = fma(g, acc, rs);
      if (MODE == MODE_EVAL) {
        a.Vout[s] = v;
        res = fabs(static_cast<double>(v) - static_cast<double>(c));
      } else {
        const double r = static_cast<double>(v) - static_cast<double>(c);
        a.r_out[s] = static_cast<float>(r);
        res = fabs(r);
      }
    }
  }
  block_max_to_slot(res, a.res_slot);
  if (MODE == MODE_GREEDY && a.change_count) block_sum_to_counter(changed, a.change_count);
}

template <typename T, int N>
static void launch_stencil_n(const StencilArgs<T>& a, int mode, hipStream_t st) {
  const dim3 grid(a.nblocks), block(kBlock);
  const size_t sh = (mode == MODE_EVAL || mode == MODE_RESID)
                        ? sizeof(T) * static_cast<size_t>(a.A) * (2 * N + 1)
                        : 0;
  switch (mode) {
    case MODE_MAX: hipLaunchKernelGGL((stencil_kernel<T, N, MODE_MAX>), grid, block, sh, st, a); break;
    case MODE_GREEDY: hipLaunchKernelGGL((stencil_kernel<T, N, MODE_GREEDY>), grid, block, sh, st, a); break;
    case MODE_EVAL: hipLaunchKernelGGL((stencil_kernel<T, N, MODE_EVAL>), grid, block, sh, st, a); break;
    default: hipLaunchKernelGGL((stencil_kernel<T, N, MODE_RESID>), grid, block, sh, st, a); break;
  }
}

template <typename T>
void launch_stencil(const StencilArgs<T>& a, int mode, hipStream_t st) {
  switch (a.g.n) {
    case 1: launch_stencil_n<T, 1>(a, mode, st); break;
    case 2: launch_stencil_n<T, 2>(a, mode, st); break;
    case 3: launch_stencil_n<T, 3>(a, mode, st); break;
    case 4: launch_stencil_n<T, 4>(a, mode, st); break;
    case 5: launch_stencil_n<T, 5>(a, mode, st); break;
    case 6: launch_stencil_n<T, 6>(a, mode, st); break;
    case 7: launch_stencil_n<T, 7>(a, mode, st); break;
    default: launch_stencil_n<T, 8>(a, mode, st); break;
  }
}

template void launch_stencil<double>(const StencilArgs<double>&, int, hipStream_t);
template void launch_stencil<float>(const StencilArgs<float>&, int, hipStream_t);

}  // namespace cpm

// K1: Bellman backup for factors that are identities or clamped +-1 shifts.
//
// With every rank term of the form I (x) ... (x) shift (x) ... (x) I, the mode
// products of V with the factors reduce to reading V at the state itself or
// at one axis neighbour (clamped at the grid edge: a move off the grid stays
// put).  Terms of one action that read the same neighbour are summed into one
// weight, so an action is a (2n+1)-point weighted stencil:
//     (P_a V)(s) = sum_p w[a][p] V(nbr_p(s)),   w[a][p] = sum of lambda_{a,r}
// over the terms whose shift is point p.  When every action a = 2k + d
// differs from a shared weight vector wbase only at the centre and its own
// axis-k points (an axis move whose slip is the same for all actions, as in
// the slip GridWorld), the shared part is applied once per state and each
// action costs 3 FMAs: 2n+1 + 3A instead of A(2n+1).  The weights then ride
// in the kernel arguments, which are scalar-loaded into SGPRs.
//
// Work layout: a persistent grid (at most 8 blocks per CU); block b owns one
// contiguous range of states, numbered so that each XCD walks a contiguous
// eighth of the state space (neighbours then share that XCD's L2).  With
// VEC = 4 a thread owns 4 consecutive states along the last dimension (needs
// m_last % 4 == 0): one coordinate decode and vector loads per 4 states, the
// last-dim neighbours come from the same vector.  The sweep reads V, R and
// the terminal bit and writes V' (and pi): 3 words + 1 bit per state.
// The max / argmax over actions (Eq. 1) and the block-reduced sup-norm
// residual are fused.
#include "common.cuh"

namespace cpm {

template <typename T, int VEC>
struct VecOf;
template <>
struct VecOf<float, 4> { using type = float4; };
template <>
struct VecOf<double, 4> { using type = double4; };

template <typename T>
__device__ __forceinline__ T comp(const typename VecOf<T, 4>::type& v, int q) {
  return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}

template <typename T>
__device__ __forceinline__ T tnanmax(T a, T b) {
  return (a != a || a > b) ? a : b;
}

// Per-state epilogue shared by both layouts.  nb: the 2N+1 stencil values.
//   AXIS: action a = 2k + d moves along axis k; its weights differ from the
//         shared base only at the centre and the two axis-k points, so
//         (P_a V)(s) = base(s) + sum of 3 terms (the slip GridWorld and any
//         model whose slip is the same for every action have this form).
//   otherwise: the full (2N+1)-point sum per action.
template <typename T, int N, int MODE, bool AXIS>
__device__ __forceinline__ void stencil_state(const StencilArgs<T>& a, const T* wsh,
                                              const T (&nb)[2 * N + 1], T rs, bool term,
                                              int pold, T tol, T& out, int& pnew, T& res,
                                              unsigned& changed) {
  constexpr int P = 2 * N + 1;
  const T g = term ? T(0) : a.gamma;
  const T c = nb[0];
  if (MODE == MODE_MAX || MODE == MODE_GREEDY) {
    T best = -INFINITY, qold = -INFINITY;
    int bi = 0;
    auto visit = [&](int act, T acc) {
      if (MODE == MODE_MAX) {
        best = fmax(best, acc);   // NaN in V still shows in the residual via c
      } else {
        const T q = fma(g, acc, rs);
        tie_update(q, act, tol, best, bi);
        if (act == pold) qold = q;
      }
    };
    if (AXIS) {
      T base = T(0);
#pragma unroll
      for (int p = 0; p < P; ++p) base = fma(a.kw_base[p], nb[p], base);
#pragma unroll
      for (int act = 0; act < 2 * N; ++act) {
        const int k = act >> 1;
        const T* w3 = a.kw_axis + 3 * act;
        T acc = fma(w3[0], nb[0], base);
        acc = fma(w3[1], nb[1 + 2 * k], acc);
        acc = fma(w3[2], nb[2 + 2 * k], acc);
        visit(act, acc);
      }
    } else {
      for (int act = 0; act < a.A; ++act) {
        const T* wa = a.w + act * P;
        T acc = T(0);
#pragma unroll
        for (int p = 0; p < P; ++p) acc = fma(wa[p], nb[p], acc);
        visit(act, acc);
      }
    }
    if (MODE == MODE_MAX) {
      out = fma(g, best, rs);
    } else {
      pnew = bi;
      if (pold >= 0 && qold >= best - tol) pnew = pold;
      changed += (pold >= 0 && pnew != pold) ? 1u : 0u;
      out = best;
    }
  } else {
    const T* wa = wsh + pold * P;
    T acc = T(0);
#pragma unroll
    for (int p = 0; p < P; ++p) acc = fma(wa[p], nb[p], acc);
    out = fma(g, acc, rs);
  }
  if (MODE != MODE_RESID) res = tnanmax(res, fabs(out - c));
}

template <typename T, int N, int MODE, int VEC, bool AXIS>
__global__ __launch_bounds__(kBlock) void stencil_kernel(StencilArgs<T> a) {
  constexpr int P = 2 * N + 1;
  extern __shared__ unsigned char smem_raw[];
  T* wsh = reinterpret_cast<T*>(smem_raw);
  if (MODE == MODE_EVAL || MODE == MODE_RESID) {
    const int nw = a.A * P;
    for (int i = threadIdx.x; i < nw; i += blockDim.x) wsh[i] = a.w[i];
    __syncthreads();
  }
  T tol = T(0);
  if (MODE == MODE_GREEDY) tol = static_cast<T>(tie_tol(a.vmax_bits));
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t s_begin = static_cast<int64_t>(blk) * a.states_per_block;
  const int64_t s_end0 = s_begin + a.states_per_block;
  const int s_end = static_cast<int>(s_end0 < a.g.S ? s_end0 : a.g.S);
  T res = T(0);
  double res_d = 0.0;   // RESID: the residual is taken in FP64
  unsigned changed = 0;
  const int mlast = a.g.size[N - 1];

  for (int s = static_cast<int>(s_begin) + threadIdx.x * VEC; s < s_end; s += kBlock * VEC) {
    int idx[N];
    uint32_t rem = static_cast<uint32_t>(s);
#pragma unroll
    for (int k = N - 1; k > 0; --k) {
      const uint32_t q = fdiv(rem, a.g.div[k]);
      idx[k] = static_cast<int>(rem - q * static_cast<uint32_t>(a.g.size[k]));
      rem = q;
    }
    idx[0] = static_cast<int>(rem);

    if (VEC == 1) {
      T nb[P];
      const T c = a.V[s];
      nb[0] = c;
#pragma unroll
      for (int k = 0; k < N; ++k) {
        // clamped moves: at the edge the neighbour is the state itself, so
        // the load address is clamped and every load is unconditional
        const int st = a.g.stride[k];
        nb[1 + 2 * k] = a.V[s + ((idx[k] < a.g.size[k] - 1) ? st : 0)];
        nb[2 + 2 * k] = a.V[s - ((idx[k] > 0) ? st : 0)];
      }
      const bool term = is_terminal(a.term_bits, s);
      const int pold = (MODE == MODE_MAX) ? -1 : (a.pi_in ? a.pi_in[s] : -1);
      T out;
      int pnew = 0;
      stencil_state<T, N, MODE, AXIS>(a, wsh, nb, a.R[s], term, pold, tol, out, pnew, res,
                                      changed);
      if (MODE == MODE_RESID) {
        const double d = static_cast<double>(out) - static_cast<double>(c);
        a.r_out[s] = static_cast<float>(d);
        res_d = nanmax(res_d, fabs(d));
      } else {
        if (a.Vout) a.Vout[s] = out;
        if (MODE == MODE_GREEDY && a.pi_out) a.pi_out[s] = pnew;
      }
    } else {
      using V4 = typename VecOf<T, 4>::type;
      const V4 c4 = *reinterpret_cast<const V4*>(a.V + s);
      V4 plus4[N > 1 ? N - 1 : 1], minus4[N > 1 ? N - 1 : 1];
#pragma unroll
      for (int k = 0; k < N - 1; ++k) {
        const int st = a.g.stride[k];
        plus4[k] = *reinterpret_cast<const V4*>(a.V + s + ((idx[k] < a.g.size[k] - 1) ? st : 0));
        minus4[k] = *reinterpret_cast<const V4*>(a.V + s - ((idx[k] > 0) ? st : 0));
      }
      const int il = idx[N - 1];
      const T left = a.V[s - ((il > 0) ? 1 : 0)];
      const T right = a.V[s + ((il + 4 < mlast) ? 4 : 3)];
      const V4 r4 = *reinterpret_cast<const V4*>(a.R + s);
      const uint32_t tw = a.term_bits[s >> 5] >> (s & 31);
      int4 p4 = make_int4(-1, -1, -1, -1);
      if (MODE != MODE_MAX && a.pi_in) p4 = *reinterpret_cast<const int4*>(a.pi_in + s);
      T outv[4];
      int pnv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T nb[P];
        nb[0] = comp<T>(c4, q);
#pragma unroll
        for (int k = 0; k < N - 1; ++k) {
          nb[1 + 2 * k] = comp<T>(plus4[k], q);
          nb[2 + 2 * k] = comp<T>(minus4[k], q);
        }
        nb[1 + 2 * (N - 1)] = q < 3 ? comp<T>(c4, q + 1) : right;
        nb[2 + 2 * (N - 1)] = q > 0 ? comp<T>(c4, q - 1) : left;
        const int pold = q == 0 ? p4.x : (q == 1 ? p4.y : (q == 2 ? p4.z : p4.w));
        pnv[q] = 0;
        stencil_state<T, N, MODE, AXIS>(a, wsh, nb, comp<T>(r4, q), (tw >> q) & 1u, pold, tol,
                                        outv[q], pnv[q], res, changed);
      }
      if (MODE == MODE_RESID) {
        float4 r;
        double d[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          d[q] = static_cast<double>(outv[q]) - static_cast<double>(comp<T>(c4, q));
          res_d = nanmax(res_d, fabs(d[q]));
        }
        r.x = static_cast<float>(d[0]);
        r.y = static_cast<float>(d[1]);
        r.z = static_cast<float>(d[2]);
        r.w = static_cast<float>(d[3]);
        *reinterpret_cast<float4*>(a.r_out + s) = r;
      } else {
        if (a.Vout) {
          V4 o;
          o.x = outv[0];
          o.y = outv[1];
          o.z = outv[2];
          o.w = outv[3];
          *reinterpret_cast<V4*>(a.Vout + s) = o;
        }
        if (MODE == MODE_GREEDY && a.pi_out)
          *reinterpret_cast<int4*>(a.pi_out + s) = make_int4(pnv[0], pnv[1], pnv[2], pnv[3]);
      }
    }
  }
  block_max_to_slot(MODE == MODE_RESID ? res_d : static_cast<double>(res), a.res_slot);
  if (MODE == MODE_GREEDY && a.change_count) block_sum_to_counter(changed, a.change_count);
}

template <typename T, int N, int VEC>
static void launch_stencil_nv(const StencilArgs<T>& a, int mode, hipStream_t st) {
  const dim3 grid(a.nblocks), block(kBlock);
  const size_t sh = (mode == MODE_EVAL || mode == MODE_RESID)
                        ? sizeof(T) * static_cast<size_t>(a.A) * (2 * N + 1)
                        : 0;
  switch (mode) {
    case MODE_MAX:
      if (a.axis) hipLaunchKernelGGL((stencil_kernel<T, N, MODE_MAX, VEC, true>), grid, block, sh, st, a);
      else hipLaunchKernelGGL((stencil_kernel<T, N, MODE_MAX, VEC, false>), grid, block, sh, st, a);
      break;
    case MODE_GREEDY:
      if (a.axis) hipLaunchKernelGGL((stencil_kernel<T, N, MODE_GREEDY, VEC, true>), grid, block, sh, st, a);
      else hipLaunchKernelGGL((stencil_kernel<T, N, MODE_GREEDY, VEC, false>), grid, block, sh, st, a);
      break;
    case MODE_EVAL: hipLaunchKernelGGL((stencil_kernel<T, N, MODE_EVAL, VEC, false>), grid, block, sh, st, a); break;
    default: hipLaunchKernelGGL((stencil_kernel<T, N, MODE_RESID, VEC, false>), grid, block, sh, st, a); break;
  }
}

template <typename T, int N>
static void launch_stencil_n(const StencilArgs<T>& a, int mode, hipStream_t st) {
  if (a.vec == 4) launch_stencil_nv<T, N, 4>(a, mode, st);
  else launch_stencil_nv<T, N, 1>(a, mode, st);
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

// K1: Bellman backup of one instance whose factors are identities or clamped
// +-1 shifts (the per-state work is in stencil_core.cuh).
//
// When every action a = 2k + d differs from a shared weight vector only at
// the centre and its own axis-k points (an axis move whose slip is the same
// for all actions, as in the slip GridWorld), the shared part is applied once
// per state and each action costs 3 FMAs: 2n+1 + 3A instead of A(2n+1).  The
// weights then ride in the kernel arguments, which are scalar-loaded into
// SGPRs.
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
#include "stencil_core.cuh"

namespace cpm {

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
  const StencilW<T> W{a.kw_base, a.kw_axis, a.w, wsh, a.A, a.gamma};
  const StencilIO<T> io{a.V, a.Vout, a.R, a.term_bits, a.pi_in, a.pi_out, a.r_out, a.obs};
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t s_begin = static_cast<int64_t>(blk) * a.states_per_block;
  const int64_t s_end0 = s_begin + a.states_per_block;
  const int s_end = static_cast<int>(s_end0 < a.g.S ? s_end0 : a.g.S);
  T res = T(0);
  double res_d = 0.0;   // RESID: the residual is taken in FP64
  unsigned changed = 0;
  // The first chunk is computed unconditionally (a thread past the block's
  // end recomputes its last chunk and stores nothing): with no bounds branch
  // before it, the kernel-argument loads and the first global loads are issued
  // together instead of in dependent rounds.
  const int s_first = static_cast<int>(s_begin) + threadIdx.x * VEC;
  const int s_last = s_end - VEC;
  stencil_chunk<T, N, MODE, VEC, AXIS>(a.g, io, W, min(s_first, s_last), tol, res, res_d, changed,
                                       s_first <= s_last);
  for (int s = s_first + kBlock * VEC; s < s_end; s += kBlock * VEC)
    stencil_chunk<T, N, MODE, VEC, AXIS>(a.g, io, W, s, tol, res, res_d, changed);
  if constexpr (MODE == MODE_RESID) {
    if (a.res_part) block_max_store(res_d, a.res_part + blk);
    else block_max_to_slot(res_d, a.res_slot);
  } else {
    if (a.res_part) block_max_store(res, a.res_part + blk);
    else block_max_to_slot(res, a.res_slot);
  }
  if (MODE == MODE_GREEDY && a.change_count) block_sum_to_counter(changed, a.change_count);
}

// Marching form for large grids (n >= 2, m_last % 4 == 0): the state space
// is a stack of m_0 planes (fixed i_0, S / m_0 contiguous states).  Block b
// owns a tile of 4 * kBlock consecutive plane offsets and walks a segment of
// planes in order, keeping the previous, current and next plane's values of
// its tile in registers, so each value is read from HBM about once per sweep
// (the one-launch form reads the dim-0 neighbours of every state again,
// S / m_0 states away).  Neighbours along the other dims are loaded and hit
// the caches (adjacent tiles run on the same XCD at the same time).
template <typename T, int N, int MODE, bool AXIS>
__global__ __launch_bounds__(kBlock) void stencil_march_kernel(StencilArgs<T> a) {
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
  const StencilW<T> W{a.kw_base, a.kw_axis, a.w, wsh, a.A, a.gamma};
  const StencilIO<T> io{a.V, a.Vout, a.R, a.term_bits, a.pi_in, a.pi_out, a.r_out, a.obs};
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int tile = lb % a.march_tiles, seg = lb / a.march_tiles;
  const int i_begin = seg * a.march_seg;
  const int i_end = min(i_begin + a.march_seg, a.g.size[0]);
  T res = T(0);
  double res_d = 0.0;
  unsigned changed = 0;
  march_column<T, N, MODE, AXIS>(a.g, io, W, tile * (kBlock * 4) + threadIdx.x * 4, i_begin, i_end,
                                 tol, res, res_d, changed);
  if constexpr (MODE == MODE_RESID) {
    if (a.res_part) block_max_store(res_d, a.res_part + lb);
    else block_max_to_slot(res_d, a.res_slot);
  } else {
    if (a.res_part) block_max_store(res, a.res_part + lb);
    else block_max_to_slot(res, a.res_slot);
  }
  if (MODE == MODE_GREEDY && a.change_count) block_sum_to_counter(changed, a.change_count);
}

template <typename T, int N>
static void launch_march_n(const StencilArgs<T>& a, int mode, hipStream_t st,
                           const LaunchTiming* tm) {
  if constexpr (N >= 2) {
    const dim3 grid(a.nblocks), block(kBlock);
    const size_t sh = (mode == MODE_EVAL || mode == MODE_RESID)
                          ? sizeof(T) * static_cast<size_t>(a.A) * (2 * N + 1)
                          : 0;
    switch (mode) {
      case MODE_MAX:
        if (a.axis) klaunch(stencil_march_kernel<T, N, MODE_MAX, true>, grid, block, sh, st, tm, a);
        else klaunch(stencil_march_kernel<T, N, MODE_MAX, false>, grid, block, sh, st, tm, a);
        break;
      case MODE_GREEDY:
        if (a.axis) klaunch(stencil_march_kernel<T, N, MODE_GREEDY, true>, grid, block, sh, st, tm, a);
        else klaunch(stencil_march_kernel<T, N, MODE_GREEDY, false>, grid, block, sh, st, tm, a);
        break;
      case MODE_EVAL: klaunch(stencil_march_kernel<T, N, MODE_EVAL, false>, grid, block, sh, st, tm, a); break;
      default: klaunch(stencil_march_kernel<T, N, MODE_RESID, false>, grid, block, sh, st, tm, a); break;
    }
  }
}

template <typename T, int N, int VEC>
static void launch_stencil_nv(const StencilArgs<T>& a, int mode, hipStream_t st,
                              const LaunchTiming* tm) {
  const dim3 grid(a.nblocks), block(kBlock);
  const size_t sh = (mode == MODE_EVAL || mode == MODE_RESID)
                        ? sizeof(T) * static_cast<size_t>(a.A) * (2 * N + 1)
                        : 0;
  switch (mode) {
    case MODE_MAX:
      if (a.axis) klaunch(stencil_kernel<T, N, MODE_MAX, VEC, true>, grid, block, sh, st, tm, a);
      else klaunch(stencil_kernel<T, N, MODE_MAX, VEC, false>, grid, block, sh, st, tm, a);
      break;
    case MODE_GREEDY:
      if (a.axis) klaunch(stencil_kernel<T, N, MODE_GREEDY, VEC, true>, grid, block, sh, st, tm, a);
      else klaunch(stencil_kernel<T, N, MODE_GREEDY, VEC, false>, grid, block, sh, st, tm, a);
      break;
    case MODE_EVAL: klaunch(stencil_kernel<T, N, MODE_EVAL, VEC, false>, grid, block, sh, st, tm, a); break;
    default: klaunch(stencil_kernel<T, N, MODE_RESID, VEC, false>, grid, block, sh, st, tm, a); break;
  }
}

template <typename T, int N>
static void launch_stencil_n(const StencilArgs<T>& a, int mode, hipStream_t st,
                             const LaunchTiming* tm) {
  if (a.march) launch_march_n<T, N>(a, mode, st, tm);
  else if (a.vec == 4) launch_stencil_nv<T, N, 4>(a, mode, st, tm);
  else launch_stencil_nv<T, N, 1>(a, mode, st, tm);
}

template <typename T>
void launch_stencil(const StencilArgs<T>& a, int mode, hipStream_t st, const LaunchTiming* tm) {
  switch (a.g.n) {
    case 1: launch_stencil_n<T, 1>(a, mode, st, tm); break;
    case 2: launch_stencil_n<T, 2>(a, mode, st, tm); break;
    case 3: launch_stencil_n<T, 3>(a, mode, st, tm); break;
    case 4: launch_stencil_n<T, 4>(a, mode, st, tm); break;
    case 5: launch_stencil_n<T, 5>(a, mode, st, tm); break;
    case 6: launch_stencil_n<T, 6>(a, mode, st, tm); break;
    case 7: launch_stencil_n<T, 7>(a, mode, st, tm); break;
    default: launch_stencil_n<T, 8>(a, mode, st, tm); break;
  }
}

template void launch_stencil<double>(const StencilArgs<double>&, int, hipStream_t,
                                     const LaunchTiming*);
template void launch_stencil<float>(const StencilArgs<float>&, int, hipStream_t,
                                    const LaunchTiming*);

}  // namespace cpm

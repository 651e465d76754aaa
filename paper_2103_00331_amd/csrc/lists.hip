// K9: Bellman backup of an MDP given directly by the per-state successor
// lists of Def. 3 (components (s, s', P(s'|s,a)) with P > 0; no Kronecker
// structure):
//     Q_a(s) = R(s) + gamma (1 - tau(s)) sum_{s'} P(s'|s,a) V(s'),
// fused with the max / argmax over actions of Eq. 1, the fixed-policy value
// (evaluation sweeps) or the FP64 policy residual.
//
// Layout: sliced ELL with 64-state slices.  The 64 states of slice q are the
// 64 lanes of one wave; for each action the slice stores as many columns as
// its longest list, column-major (entry j of lane l at (c0 + j) * 64 + l,
// padded with probability 0).  A column load is 64 consecutive words
// (coalesced) and the column ranges are the same for the whole wave, so they
// are read through the scalar unit.  Each block walks a contiguous range of
// slices (blocks numbered XCD-contiguously), so the successors a wave
// gathers, which sit near its own states in most models, are shared through
// that XCD's L2.
#include "common.cuh"

namespace cpm {

template <typename T>
__device__ __forceinline__ T lnanmax(T a, T b) {
  return (a != a || a > b) ? a : b;
}

template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void lists_kernel(ListsArgs<T> a) {
  constexpr int kWaves = kBlock / kSlice;
  T tol = T(0);
  if (MODE == MODE_GREEDY) tol = static_cast<T>(tie_tol(a.vmax_bits));
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int lane = threadIdx.x & (kSlice - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kSlice);
  const int q_begin = blk * a.slices_per_block;
  const int q_end = min(q_begin + a.slices_per_block, a.nslices);
  T res = T(0);
  double res_d = 0.0;
  unsigned changed = 0;
  for (int q = q_begin + wave; q < q_end; q += kWaves) {
    const int s = q * kSlice + lane;
    const bool live = s < a.S;
    const int sc = live ? s : a.S - 1;
    const T c = a.V[sc];
    const T rs = a.R[sc];
    const T g = is_terminal(a.term_bits, sc) ? T(0) : a.gamma;
    const int32_t* cp = a.col_ptr + static_cast<size_t>(q) * a.A;
    T out;
    int pnew = 0;
    if (MODE == MODE_MAX || MODE == MODE_GREEDY) {
      const int pold = (MODE == MODE_GREEDY && a.pi_in) ? a.pi_in[sc] : -1;
      T best = -INFINITY, qold = -INFINITY;
      int bi = 0;
      int c0 = cp[0];
      for (int act = 0; act < a.A; ++act) {
        const int c1 = cp[act + 1];
        T acc = T(0);
        for (int col = c0; col < c1; ++col) {
          const size_t e = static_cast<size_t>(col) * kSlice + lane;
          acc = fma(a.prob[e], a.V[a.succ[e]], acc);
        }
        c0 = c1;
        if (MODE == MODE_MAX) {
          best = fmax(best, acc);   // a NaN in V still shows in the residual via c
        } else {
          const T qv = fma(g, acc, rs);
          tie_update(qv, act, tol, best, bi);
          if (act == pold) qold = qv;
        }
      }
      if (MODE == MODE_MAX) {
        out = fma(g, best, rs);
      } else {
        pnew = bi;
        if (pold >= 0 && qold >= best - tol) pnew = pold;
        if (live) changed += (pold >= 0 && pnew != pold) ? 1u : 0u;
        out = best;
      }
    } else {
      // fixed policy: the lane's own action (columns differ across lanes)
      const int act = a.pi_in[sc];
      T acc = T(0);
      for (int col = cp[act]; col < cp[act + 1]; ++col) {
        const size_t e = static_cast<size_t>(col) * kSlice + lane;
        acc = fma(a.prob[e], a.V[a.succ[e]], acc);
      }
      out = fma(g, acc, rs);
    }
    if (!live) continue;
    if (MODE == MODE_RESID) {
      const double d = static_cast<double>(out) - static_cast<double>(c);
      a.r_out[s] = static_cast<float>(d);
      res_d = nanmax(res_d, fabs(d));
    } else {
      res = lnanmax(res, static_cast<T>(fabs(out - c)));
      if (a.Vout) a.Vout[s] = out;
      if (MODE == MODE_GREEDY && a.pi_out) a.pi_out[s] = pnew;
    }
  }
  if constexpr (MODE == MODE_RESID) {
    if (a.res_part) block_max_store(res_d, a.res_part + blk);
    else block_max_to_slot(res_d, a.res_slot);
  } else {
    if (a.res_part) block_max_store(res, a.res_part + blk);
    else block_max_to_slot(res, a.res_slot);
  }
  if (MODE == MODE_GREEDY && a.change_count) block_sum_to_counter(changed, a.change_count);
}

template <typename T>
void launch_lists(const ListsArgs<T>& a, int mode, hipStream_t st, const LaunchTiming* tm) {
  const dim3 grid(a.nblocks), block(kBlock);
  switch (mode) {
    case MODE_MAX: klaunch(lists_kernel<T, MODE_MAX>, grid, block, 0, st, tm, a); break;
    case MODE_GREEDY: klaunch(lists_kernel<T, MODE_GREEDY>, grid, block, 0, st, tm, a); break;
    case MODE_EVAL: klaunch(lists_kernel<T, MODE_EVAL>, grid, block, 0, st, tm, a); break;
    default: klaunch(lists_kernel<T, MODE_RESID>, grid, block, 0, st, tm, a); break;
  }
}

template void launch_lists<double>(const ListsArgs<double>&, int, hipStream_t,
                                   const LaunchTiming*);
template void launch_lists<float>(const ListsArgs<float>&, int, hipStream_t,
                                  const LaunchTiming*);

}  // namespace cpm

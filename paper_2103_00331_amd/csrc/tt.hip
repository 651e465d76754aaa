// K10: Bellman backup for Tensor-Train transition models (the matrix-product
// operators that Sec. 5 names beside the CP form; Tucker operators arrive
// here rewritten as Tensor-Trains at create).  Action a has cores G_k of
// shape [b_k, m_k, m_k, b_{k+1}], b_0 = b_n = 1, and
//     P_a[s, s'] = G_0[:, s_0, s'_0, :] G_1[:, s_1, s'_1, :] ... G_{n-1}[...].
// Applied to V this is a chain of bonded mode products, last dimension
// first: X^{(n)} = V (one channel), and for k = n-1 .. 0
//     X^{(k)}[l][.., i_k, ..] = sum_{r < b_{k+1}} sum_j G_k[l, i_k, j, r] X^{(k+1)}[r][.., j, ..],
// with one S-sized channel per bond value l < b_k.  X^{(0)} = P_a V.
//
// One launch per (action, dimension) streams X^{(k+1)} (b_{k+1} channels)
// to X^{(k)} (b_k channels): for each fiber position (all coordinates but
// i_k) it is a small matrix product (b_k m_k) x (b_{k+1} m_k), i.e. a GEMM
// over the S / m_k fiber positions.  With m_k = 16 and a fiber stride that
// is a multiple of 16 it runs on the matrix cores (16 positions per matrix
// tile, the cores held in registers for the whole launch); otherwise on the
// vector ALUs with the cores read as wave-uniform scalars.  The last launch
// of each action writes Y[a] = P_a V; one epilogue kernel then fuses Eq. 1:
// the max / argmax over actions, the fixed-policy value or the FP64 policy
// residual, and the sup-norm residual.
//
// Device core layout, per (action, k): Gd[r][j][l][i] with i, j padded to
// MM (4, 8 or 16, the smallest >= m_k) and l padded to a multiple of 4,
// zeros in the padding, so that every kernel reads whole unguarded blocks.
#include "common.cuh"

namespace cpm {

typedef float tt_f4 __attribute__((ext_vector_type(4)));
typedef double tt_d4 __attribute__((ext_vector_type(4)));

template <typename T>
struct TTAcc;
template <>
struct TTAcc<float> { using type = tt_f4; };
template <>
struct TTAcc<double> { using type = tt_d4; };

// One 16 x 16 x 4 matrix product.  Lane (g, c) = (lane / 16, lane % 16)
// supplies A[i = c][k = g] and B[k = g][n = c]; the result register r holds
// D[i = 4g + r][n = c] (FP32) or D[i = g + 4r][n = c] (FP64).
__device__ __forceinline__ tt_f4 tt_mfma(float a, float b, tt_f4 acc) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
}
__device__ __forceinline__ tt_d4 tt_mfma(double a, double b, tt_d4 acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
}

// Vector-ALU bonded mode product.  Thread = one fiber position, BO output
// channels (blockIdx.y selects the group of BO), all input channels.
template <typename T, int MM, int BO>
__global__ __launch_bounds__(kBlock) void tt_step_vec(TTStepArgs<T> a) {
  const unsigned upos = blockIdx.x * kBlock + threadIdx.x;
  if (upos >= static_cast<unsigned>(a.positions)) return;
  const int pos = static_cast<int>(upos);
  const int l0 = blockIdx.y * BO;
  const int p = static_cast<int>(fdiv(static_cast<uint32_t>(pos), a.post_div));
  const int q = pos - p * a.post;
  const int base = p * a.m * a.post + q;
  T acc[BO][MM];
#pragma unroll
  for (int b = 0; b < BO; ++b)
#pragma unroll
    for (int i = 0; i < MM; ++i) acc[b][i] = T(0);
  for (int r = 0; r < a.b_in; ++r) {
    const T* __restrict__ src = a.in + static_cast<size_t>(r) * a.S + base;
    T x[MM];
#pragma unroll
    for (int j = 0; j < MM; ++j) x[j] = j < a.m ? src[j * a.post] : T(0);
    const T* __restrict__ G = a.core + static_cast<size_t>(r) * MM * a.lpad * MM;
#pragma unroll
    for (int j = 0; j < MM; ++j)
#pragma unroll
      for (int b = 0; b < BO; ++b)
#pragma unroll
        for (int i = 0; i < MM; ++i)
          acc[b][i] = fma(G[(j * a.lpad + l0 + b) * MM + i], x[j], acc[b][i]);
  }
#pragma unroll
  for (int b = 0; b < BO; ++b) {
    if (l0 + b >= a.b_out) break;
    T* __restrict__ dst = a.out + static_cast<size_t>(l0 + b) * a.S + base;
#pragma unroll
    for (int i = 0; i < MM; ++i)
      if (i < a.m) dst[i * a.post] = acc[b][i];
  }
}

// Matrix-core bonded mode product for m_k = 16 and a fiber stride (post)
// that is a multiple of 16: a tile of 16 consecutive fiber positions shares
// its leading coordinates, so lane (g, c) reads X[r][base_c + (4q + g) post]
// for k-block (r, q) -- 16 consecutive words per lane group -- and writes
// its result rows the same way.  The A operands (the cores of BO output
// channels, BI >= b_in input channels) stay in registers; each wave walks
// tiles with a grid stride.
template <typename T, int BO, int BI>
__global__ __launch_bounds__(kBlock) void tt_step_mfma(TTStepArgs<T> a) {
  using Acc = typename TTAcc<T>::type;
  constexpr bool f64 = sizeof(T) == 8;
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, g = lane >> 4;
  const int l0 = blockIdx.y * BO;
  T aw[BO][BI][4];
#pragma unroll
  for (int b = 0; b < BO; ++b)
#pragma unroll
    for (int r = 0; r < BI; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        aw[b][r][q] = r < a.b_in ? a.core[((r * 16 + 4 * q + g) * a.lpad + l0 + b) * 16 + c]
                                 : T(0);
  const int ntiles = a.positions >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(
      xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6));
  const int nwaves = gridDim.x * (kBlock / 64);
  for (int t = wave; t < ntiles; t += nwaves) {
    const int pos = t * 16 + c;
    const int p = static_cast<int>(fdiv(static_cast<uint32_t>(pos), a.post_div));
    const int base = p * 16 * a.post + (pos - p * a.post);
    T x[BI][4];
#pragma unroll
    for (int r = 0; r < BI; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        x[r][q] = r < a.b_in ? a.in[static_cast<size_t>(r) * a.S + base + (4 * q + g) * a.post]
                             : T(0);
#pragma unroll
    for (int b = 0; b < BO; ++b) {
      if (l0 + b >= a.b_out) break;
      Acc acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int r = 0; r < BI; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc = tt_mfma(aw[b][r][q], x[r][q], acc);
      T* __restrict__ dst = a.out + static_cast<size_t>(l0 + b) * a.S + base;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) dst[(f64 ? g + 4 * rr : 4 * g + rr) * a.post] = acc[rr];
    }
  }
}

// Eq. 1 over Y[a] = P_a V (a < A): Q_a(s) = R(s) + gamma (1 - tau(s)) Y[a](s).
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void tt_epilogue(TTEpiArgs<T> a) {
  T tol = T(0);
  if (MODE == MODE_GREEDY) tol = static_cast<T>(tie_tol(a.vmax_bits));
  T res = T(0);
  double res_d = 0.0;
  unsigned changed = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t s = blockIdx.x * kBlock + threadIdx.x; s < a.S; s += stride) {
    const T c = a.V[s];
    const T rs = a.R[s];
    const T gm = is_terminal(a.term_bits, static_cast<int>(s)) ? T(0) : a.gamma;
    T out;
    int pnew = 0;
    if (MODE == MODE_MAX) {
      T best = -INFINITY;
      for (int act = 0; act < a.A; ++act)
        best = fmax(best, a.Y[static_cast<size_t>(act) * a.S + s]);   // a NaN in V shows via c
      out = fma(gm, best, rs);
    } else if (MODE == MODE_GREEDY) {
      const int pold = a.pi_in ? a.pi_in[s] : -1;
      T best = -INFINITY, qold = -INFINITY;
      int bi = 0;
      for (int act = 0; act < a.A; ++act) {
        const T qv = fma(gm, a.Y[static_cast<size_t>(act) * a.S + s], rs);
        tie_update(qv, act, tol, best, bi);
        if (act == pold) qold = qv;
      }
      pnew = bi;
      if (pold >= 0 && qold >= best - tol) pnew = pold;
      changed += (pold >= 0 && pnew != pold) ? 1u : 0u;
      out = best;
    } else {
      out = fma(gm, a.Y[static_cast<size_t>(a.pi_in[s]) * a.S + s], rs);
    }
    if (MODE == MODE_RESID) {
      const double d = static_cast<double>(out) - static_cast<double>(c);
      a.r_out[s] = static_cast<float>(d);
      res_d = nanmax(res_d, fabs(d));
    } else {
      res = nanmax_t(res, static_cast<T>(fabs(out - c)));
      if (a.Vout) a.Vout[s] = out;
      if (MODE == MODE_GREEDY && a.pi_out) a.pi_out[s] = pnew;
    }
  }
  if constexpr (MODE == MODE_RESID) block_max_to_slot(res_d, a.res_slot);
  else block_max_to_slot(res, a.res_slot);
  if (MODE == MODE_GREEDY && a.change_count) block_sum_to_counter(changed, a.change_count);
}

// Which kernel runs a step.
template <typename T>
static bool step_on_mfma(const TTStepArgs<T>& a) {
  return a.mm == 16 && a.m == 16 && a.post % 16 == 0 && a.b_in >= 2 && a.b_in <= 8;
}

template <typename T, int BO>
static void launch_mfma_bi(const TTStepArgs<T>& a, dim3 grid, hipStream_t st,
                           const LaunchTiming* tm) {
  if (a.b_in <= 2) klaunch(tt_step_mfma<T, BO, 2>, grid, dim3(kBlock), 0, st, tm, a);
  else if (a.b_in <= 4) klaunch(tt_step_mfma<T, BO, 4>, grid, dim3(kBlock), 0, st, tm, a);
  else klaunch(tt_step_mfma<T, (sizeof(T) == 8 && BO > 2 ? 2 : BO), 8>, grid, dim3(kBlock), 0, st,
               tm, a);
}

template <typename T, int MM>
static void launch_vec_mm(const TTStepArgs<T>& a, hipStream_t st, const LaunchTiming* tm) {
  const int bo = a.b_out >= 4 ? 4 : (a.b_out >= 2 ? 2 : 1);
  const dim3 grid((a.positions + kBlock - 1) / kBlock, (a.b_out + bo - 1) / bo);
  if (bo == 4) klaunch(tt_step_vec<T, MM, 4>, grid, dim3(kBlock), 0, st, tm, a);
  else if (bo == 2) klaunch(tt_step_vec<T, MM, 2>, grid, dim3(kBlock), 0, st, tm, a);
  else klaunch(tt_step_vec<T, MM, 1>, grid, dim3(kBlock), 0, st, tm, a);
}

template <typename T>
void launch_tt_step(const TTStepArgs<T>& a, hipStream_t st, const LaunchTiming* tm) {
  if (step_on_mfma(a)) {
    const int bo = (sizeof(T) == 8 && a.b_in > 4) ? 2 : 4;
    const int bo_used = a.b_out >= bo ? bo : (a.b_out >= 2 ? 2 : 1);
    const int tiles = a.positions / 16;
    const int blocks = (tiles + 3) / 4 < kMaxBlocks ? (tiles + 3) / 4 : kMaxBlocks;
    const dim3 grid(blocks, (a.b_out + bo_used - 1) / bo_used);
    if (bo_used == 4) launch_mfma_bi<T, 4>(a, grid, st, tm);
    else if (bo_used == 2) launch_mfma_bi<T, 2>(a, grid, st, tm);
    else launch_mfma_bi<T, 1>(a, grid, st, tm);
    return;
  }
  switch (a.mm) {
    case 4: launch_vec_mm<T, 4>(a, st, tm); break;
    case 8: launch_vec_mm<T, 8>(a, st, tm); break;
    default: launch_vec_mm<T, 16>(a, st, tm); break;
  }
}

template <typename T>
void launch_tt_epilogue(const TTEpiArgs<T>& a, int mode, hipStream_t st, const LaunchTiming* tm) {
  const int blocks = (a.S + kBlock - 1) / kBlock < kMaxBlocks ? (a.S + kBlock - 1) / kBlock : kMaxBlocks;
  const dim3 grid(blocks), block(kBlock);
  switch (mode) {
    case MODE_MAX: klaunch(tt_epilogue<T, MODE_MAX>, grid, block, 0, st, tm, a); break;
    case MODE_GREEDY: klaunch(tt_epilogue<T, MODE_GREEDY>, grid, block, 0, st, tm, a); break;
    case MODE_EVAL: klaunch(tt_epilogue<T, MODE_EVAL>, grid, block, 0, st, tm, a); break;
    default: klaunch(tt_epilogue<T, MODE_RESID>, grid, block, 0, st, tm, a); break;
  }
}

template void launch_tt_step<double>(const TTStepArgs<double>&, hipStream_t, const LaunchTiming*);
template void launch_tt_step<float>(const TTStepArgs<float>&, hipStream_t, const LaunchTiming*);
template void launch_tt_epilogue<double>(const TTEpiArgs<double>&, int, hipStream_t,
                                         const LaunchTiming*);
template void launch_tt_epilogue<float>(const TTEpiArgs<float>&, int, hipStream_t,
                                        const LaunchTiming*);

}  // namespace cpm

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
// over the S / m_k fiber positions.  With m_k = 16 it runs on the matrix
// cores (16 positions per matrix tile, the cores held in registers for the
// whole launch, 16-byte loads and stores where the layout allows); otherwise
// on the vector ALUs with the cores read as wave-uniform scalars.  The last launch
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

// Matrix-core bonded mode products for m_k = 16.  The A operands (the cores
// of BO output channels and BI >= b_in input channels) stay in registers for
// the whole launch; each wave walks tiles of 16 fiber positions (the matrix
// columns n) with a grid stride (two waves per SIMD overlap one's loads with
// the other's matrix products).  Three layouts of a tile in memory:
//   TT_ROWS  (fiber stride post % 16 == 0): the 16 positions of a tile are
//            consecutive words of each of the 16 rows j; lane (g, c) reads
//            row j = 4q + g of position c (4-byte accesses).
//   TT_WIDE  (FP32, post % U == 0, U = 16 bytes / word): a wave step takes U
//            interleaved tiles, lane c holding U consecutive positions of
//            every row in one 16-byte load, and writes its U results of each
//            output row with one 16-byte store.
//   TT_INNER (post == 1, the last dimension): the 16 values of a fiber are
//            consecutive; lane (g, c) loads j = 4g .. 4g + 3 of fiber c in one
//            16-byte access (k-block q then holds j = 4g + q) and stores its
//            4 output rows i = 4g .. 4g + 3 the same way (FP64 results come out
//            as rows g + 4r, so the A rows are permuted to make them 4g + r).
enum { TT_ROWS = 0, TT_WIDE = 1, TT_INNER = 2 };

template <typename T>
struct TTVec;
template <>
struct TTVec<float> {
  typedef float type __attribute__((ext_vector_type(4)));
};
template <>
struct TTVec<double> {
  typedef double type __attribute__((ext_vector_type(2)));
};

template <typename T, int BO, int BI, int LAYOUT>
__global__ __launch_bounds__(kBlock) void tt_step_mfma(TTStepArgs<T> a) {
  using Acc = typename TTAcc<T>::type;
  using V16 = typename TTVec<T>::type;
  constexpr bool f64 = sizeof(T) == 8;
  constexpr int W = 16 / sizeof(T);                   // words per 16-byte access
  constexpr int U = LAYOUT == TT_WIDE ? W : 1;        // tiles per wave step
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, g = lane >> 4;
  const int l0 = blockIdx.y * BO;
  // A row held by lane c (TT_INNER, FP64: row permutation, see above)
  const int arow = (LAYOUT == TT_INNER && f64) ? 4 * (c & 3) + (c >> 2) : c;
  T aw[BO][BI][4];
#pragma unroll
  for (int b = 0; b < BO; ++b)
#pragma unroll
    for (int r = 0; r < BI; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = LAYOUT == TT_INNER ? 4 * g + q : 4 * q + g;
        aw[b][r][q] = r < a.b_in ? a.core[((r * 16 + j) * a.lpad + l0 + b) * 16 + arow] : T(0);
      }
  const int nsteps = a.positions / (16 * U);
  const int wave = __builtin_amdgcn_readfirstlane(
      xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + (threadIdx.x >> 6));
  const int nwaves = gridDim.x * (kBlock / 64);
  // TT_ROWS / TT_WIDE: offset of this lane's first position of step t, and
  // the load of a step's operands (rows j = 4q + g of every input channel)
  auto base_of = [&](int t) {
    const int pos = (t * 16 + c) * U;
    const int p = static_cast<int>(fdiv(static_cast<uint32_t>(pos), a.post_div));
    return p * 16 * a.post + (pos - p * a.post);
  };
  auto load_step = [&](int base, T (&x)[BI][4][U]) {
#pragma unroll
    for (int r = 0; r < BI; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T* src = a.in + static_cast<size_t>(r) * a.S + base + (4 * q + g) * a.post;
        if (r >= a.b_in) {
#pragma unroll
          for (int u = 0; u < U; ++u) x[r][q][u] = T(0);
        } else if constexpr (U == 1) {
          x[r][q][0] = *src;
        } else {
          const V16 v = *reinterpret_cast<const V16*>(src);
#pragma unroll
          for (int u = 0; u < U; ++u) x[r][q][u] = v[u];
        }
      }
  };
  for (int t = wave; t < nsteps; t += nwaves) {
    if constexpr (LAYOUT == TT_INNER) {
      const size_t base = static_cast<size_t>(t * 16 + c) * 16 + 4 * g;
      T x[BI][4];
#pragma unroll
      for (int r = 0; r < BI; ++r) {
        if (r < a.b_in) {
          const T* src = a.in + static_cast<size_t>(r) * a.S + base;
#pragma unroll
          for (int h = 0; h < 4; h += W) {
            const V16 v = *reinterpret_cast<const V16*>(src + h);
#pragma unroll
            for (int e = 0; e < W; ++e) x[r][h + e] = v[e];
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) x[r][q] = T(0);
        }
      }
#pragma unroll
      for (int b = 0; b < BO; ++b) {
        if (l0 + b >= a.b_out) break;
        Acc acc = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int r = 0; r < BI; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc = tt_mfma(aw[b][r][q], x[r][q], acc);
        T* dst = a.out + static_cast<size_t>(l0 + b) * a.S + base;
#pragma unroll
        for (int h = 0; h < 4; h += W) {
          V16 v;
#pragma unroll
          for (int e = 0; e < W; ++e) v[e] = acc[h + e];
          *reinterpret_cast<V16*>(dst + h) = v;
        }
      }
    } else {
      const int base = base_of(t);
      T x[BI][4][U];
      load_step(base, x);
#pragma unroll
      for (int b = 0; b < BO; ++b) {
        if (l0 + b >= a.b_out) break;
        Acc acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          acc[u] = Acc{T(0), T(0), T(0), T(0)};
#pragma unroll
          for (int r = 0; r < BI; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[u] = tt_mfma(aw[b][r][q], x[r][q][u], acc[u]);
        }
        T* dst = a.out + static_cast<size_t>(l0 + b) * a.S + base;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          T* d = dst + (f64 ? g + 4 * rr : 4 * g + rr) * a.post;
          if constexpr (U == 1) {
            *d = acc[0][rr];
          } else {
            V16 v;
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = acc[u][rr];
            *reinterpret_cast<V16*>(d) = v;
          }
        }
      }
    }
  }
}

// TT_WIDE with the input tile shared in LDS (FP32, b_in = 4): the block's
// 256 threads load a step's 64 positions x 16 rows x 4 input channels
// (16 KB) with 16-byte accesses into one of two LDS buffers while the
// previous step is multiplied out of the other; wave w computes output
// channel l0 + w alone (its core in 16 registers).  Used for b_out = 1 (the
// first dimension, which writes P_a V), where the wide kernel's one working
// wave per block waits on its own loads; for b_out = 4 the two kernels run
// at the same speed (about 46% matrix-core busy at 4.5 TB/s).
constexpr int kTTShRow = 68;         // LDS words per 64-position row (+4: bank spread)

__global__ __launch_bounds__(kBlock) void tt_step_shared(TTStepArgs<float> a) {
  __shared__ float xs[2][4 * 16 * kTTShRow];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int l = blockIdx.y * 4 + wv;                 // this wave's output channel
  const bool act = l < a.b_out;
  float aw[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      aw[r][q] = act ? a.core[((r * 16 + 4 * q + g) * a.lpad + l) * 16 + c] : 0.f;
  const int nsteps = a.positions / 64;
  // loader: thread t moves 16-byte pieces (r, j, p4) with p4 = 4-position group
  auto base_of = [&](int t, int p4) {
    const int pos = t * 64 + 4 * p4;
    const int p = static_cast<int>(fdiv(static_cast<uint32_t>(pos), a.post_div));
    return p * 16 * a.post + (pos - p * a.post);
  };
  tt_f4 stage[4];
  auto load = [&](int t) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int piece = threadIdx.x + k * kBlock;    // 1024 pieces: (r, j, p4) = (4, 16, 16)
      const int p4 = piece & 15, j = (piece >> 4) & 15, r = piece >> 8;
      stage[k] = *reinterpret_cast<const tt_f4*>(a.in + static_cast<size_t>(r) * a.S +
                                                 base_of(t, p4) + j * a.post);
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int piece = threadIdx.x + k * kBlock;
      const int p4 = piece & 15, j = (piece >> 4) & 15, r = piece >> 8;
      *reinterpret_cast<tt_f4*>(&xs[buf][(r * 16 + j) * kTTShRow + 4 * p4]) = stage[k];
    }
  };
  int t = blockIdx.x;
  if (t < nsteps) {
    load(t);
    put(0);
  }
  __syncthreads();
  int buf = 0;
  for (; t < nsteps; t += gridDim.x) {
    const int tn = t + gridDim.x;
    if (tn < nsteps) load(tn);                      // in flight during the products
    if (act) {
      tt_f4 acc[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] = tt_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const tt_f4 x = *reinterpret_cast<const tt_f4*>(&xs[buf][(r * 16 + 4 * q + g) * kTTShRow + 4 * c]);
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] = tt_mfma(aw[r][q], x[u], acc[u]);
        }
      const int base = base_of(t, c);
      float* dst = a.out + static_cast<size_t>(l) * a.S + base;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        tt_f4 v;
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = acc[u][rr];
        *reinterpret_cast<tt_f4*>(dst + (4 * g + rr) * a.post) = v;
      }
    }
    if (tn < nsteps) put(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
}

// The last two dimensions in one launch (FP32, m_{n-1} = m_{n-2} = 16, bonds
// b_{n-1}, b_{n-2} <= 4): a wave takes a block of 256 states (fixed leading
// coordinates), runs the last-dimension product as TT_INNER (16 fibers, one
// 16-byte load each), which leaves lane (g, c) with
// Y[l][j_{n-2} = c][i_{n-1} = 4g + r] for every middle bond value l, passes
// those through its own LDS slab to read them back transposed, and runs the
// dim n-2 product with the data as the A operand (rows i_{n-1}) and the core
// as the B operand (columns i_{n-2}), so that lane (g, c) ends with
// out[i_{n-2} = c][i_{n-1} = 4g .. 4g + 3] and stores it in 16 bytes.  The
// b_{n-1} intermediate channels never reach HBM.
constexpr int kTT2Row = 20;          // LDS words per 16-value row (+4: no bank conflicts)

__device__ __forceinline__ void tt_wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int BB, int BO>
__global__ __launch_bounds__(kBlock) void tt_step_last2(TTStep2Args a) {
  __shared__ float slab[kBlock / 64][BB * 16 * kTT2Row];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  float* Ys = slab[wv];
  float aw[BB][4], bw[BO][BB][4];
#pragma unroll
  for (int l = 0; l < BB; ++l)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      aw[l][q] = l < a.b_mid ? a.core1[((4 * g + q) * a.lpad1 + l) * 16 + c] : 0.f;
#pragma unroll
  for (int o = 0; o < BO; ++o)
#pragma unroll
    for (int l = 0; l < BB; ++l)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        bw[o][l][q] = (l < a.b_mid && o < a.b_out)
                          ? a.core2[((l * 16 + 4 * q + g) * a.lpad2 + o) * 16 + c] : 0.f;
  const int nblk = a.S >> 8;
  const int wave = __builtin_amdgcn_readfirstlane(
      xcd_block(blockIdx.x, gridDim.x) * (kBlock / 64) + wv);
  const int nwaves = gridDim.x * (kBlock / 64);
  for (int t = wave; t < nblk; t += nwaves) {
    const size_t base = static_cast<size_t>(t) * 256;
    const tt_f4 x = *reinterpret_cast<const tt_f4*>(a.in + base + c * 16 + 4 * g);
#pragma unroll
    for (int l = 0; l < BB; ++l) {
      if (l >= a.b_mid) break;
      tt_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) acc = tt_mfma(aw[l][q], x[q], acc);
      *reinterpret_cast<tt_f4*>(Ys + (l * 16 + c) * kTT2Row + 4 * g) = acc;
    }
    tt_wave_fence();
    float y[BB][4];
#pragma unroll
    for (int l = 0; l < BB; ++l)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        y[l][q] = l < a.b_mid ? Ys[(l * 16 + 4 * q + g) * kTT2Row + c] : 0.f;
    tt_wave_fence();     // the next block's writes come after these reads
#pragma unroll
    for (int o = 0; o < BO; ++o) {
      if (o >= a.b_out) break;
      tt_f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int l = 0; l < BB; ++l)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc = tt_mfma(y[l][q], bw[o][l][q], acc);
      *reinterpret_cast<tt_f4*>(a.out + static_cast<size_t>(o) * a.S + base + c * 16 + 4 * g) = acc;
    }
  }
}

// Eq. 1 over Y[a] = P_a V (a < A): Q_a(s) = R(s) + gamma (1 - tau(s)) Y[a](s).
// E consecutive states per thread (E = 16 bytes / word when S allows: every
// stream is then read with 16-byte loads).
template <typename T, int MODE, int E>
__global__ __launch_bounds__(kBlock) void tt_epilogue(TTEpiArgs<T> a) {
  using V16 = typename TTVec<T>::type;
  auto load = [&](const T* p, T (&v)[E]) {
    if constexpr (E == 1) {
      v[0] = *p;
    } else {
      const V16 w = *reinterpret_cast<const V16*>(p);
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = w[e];
    }
  };
  T tol = T(0);
  if (MODE == MODE_GREEDY) tol = static_cast<T>(tie_tol(a.vmax_bits));
  T res = T(0);
  double res_d = 0.0;
  unsigned changed = 0;
  const int64_t nv = a.S / E;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
  for (int64_t v = blockIdx.x * kBlock + threadIdx.x; v < nv; v += stride) {
    const int64_t s0 = v * E;
    T c[E], rs[E], gm[E], out[E];
    int pnew[E];
    load(a.V + s0, c);
    load(a.R + s0, rs);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      gm[e] = is_terminal(a.term_bits, static_cast<int>(s0 + e)) ? T(0) : a.gamma;
      pnew[e] = 0;
    }
    if (MODE == MODE_MAX) {
      T best[E];
#pragma unroll
      for (int e = 0; e < E; ++e) best[e] = -INFINITY;
      for (int act = 0; act < a.A; ++act) {
        T y[E];
        load(a.Y + static_cast<size_t>(act) * a.S + s0, y);
#pragma unroll
        for (int e = 0; e < E; ++e) best[e] = fmax(best[e], y[e]);   // a NaN in V shows via c
      }
#pragma unroll
      for (int e = 0; e < E; ++e) out[e] = fma(gm[e], best[e], rs[e]);
    } else if (MODE == MODE_GREEDY) {
      int pold[E], bi[E];
      T best[E], qold[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        pold[e] = a.pi_in ? a.pi_in[s0 + e] : -1;
        best[e] = -INFINITY;
        qold[e] = -INFINITY;
        bi[e] = 0;
      }
      for (int act = 0; act < a.A; ++act) {
        T y[E];
        load(a.Y + static_cast<size_t>(act) * a.S + s0, y);
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const T qv = fma(gm[e], y[e], rs[e]);
          tie_update(qv, act, tol, best[e], bi[e]);
          if (act == pold[e]) qold[e] = qv;
        }
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        pnew[e] = bi[e];
        if (pold[e] >= 0 && qold[e] >= best[e] - tol) pnew[e] = pold[e];
        changed += (pold[e] >= 0 && pnew[e] != pold[e]) ? 1u : 0u;
        out[e] = best[e];
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e)
        out[e] = fma(gm[e], a.Y[static_cast<size_t>(a.pi_in[s0 + e]) * a.S + s0 + e], rs[e]);
    }
    if (MODE == MODE_RESID) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const double d = static_cast<double>(out[e]) - static_cast<double>(c[e]);
        a.r_out[s0 + e] = static_cast<float>(d);
        res_d = nanmax(res_d, fabs(d));
      }
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) res = nanmax_t(res, static_cast<T>(fabs(out[e] - c[e])));
      if (a.Vout) {
        if constexpr (E == 1) {
          a.Vout[s0] = out[0];
        } else {
          V16 w;
#pragma unroll
          for (int e = 0; e < E; ++e) w[e] = out[e];
          *reinterpret_cast<V16*>(a.Vout + s0) = w;
        }
      }
      if (MODE == MODE_GREEDY && a.pi_out) {
#pragma unroll
        for (int e = 0; e < E; ++e) a.pi_out[s0 + e] = pnew[e];
      }
    }
  }
  if constexpr (MODE == MODE_RESID) block_max_to_slot(res_d, a.res_slot);
  else block_max_to_slot(res, a.res_slot);
  if (MODE == MODE_GREEDY && a.change_count) block_sum_to_counter(changed, a.change_count);
}

// Which kernel runs a step: the matrix cores when m_k = 16 and the tiles of
// one of the three layouts cover the fiber positions exactly, else the
// vector kernel.
template <typename T>
static int mfma_layout(const TTStepArgs<T>& a) {
  constexpr int W = 16 / static_cast<int>(sizeof(T));
  if (a.m != 16 || a.mm != 16 || a.b_in > 8) return -1;
  // 16-byte accesses need 16-byte aligned channels (the caller's V may not be)
  const bool al = ((reinterpret_cast<uintptr_t>(a.in) | reinterpret_cast<uintptr_t>(a.out)) & 15) == 0;
  if (a.post == 1) return (al && a.positions % 16 == 0) ? TT_INNER : -1;
  // FP64 keeps the row layout: the wide one holds half the output channels
  // per block there (registers), which reads every input twice
  if (sizeof(T) == 4 && al && a.post % W == 0 && a.positions % (16 * W) == 0) return TT_WIDE;
  if (a.post % 16 == 0) return TT_ROWS;
  return -1;
}

// Output channels per block: as many as the registers hold beside the
// operands (more input channels or wider tiles leave room for fewer).
template <typename T>
static int mfma_bo_cap(int bi, int layout) {
  if (layout == TT_WIDE) return bi == 8 ? 1 : 4;
  return bi == 8 ? 2 : 4;
}

template <typename T, int LAYOUT, int BI>
static void launch_mfma_bo(const TTStepArgs<T>& a, int bo, hipStream_t st, const LaunchTiming* tm) {
  constexpr int U = LAYOUT == TT_WIDE ? 16 / static_cast<int>(sizeof(T)) : 1;
  const int steps = a.positions / (16 * U);
  const int blocks = (steps + 3) / 4 < kMaxBlocks ? (steps + 3) / 4 : kMaxBlocks;
  const dim3 grid(blocks, (a.b_out + bo - 1) / bo), block(kBlock);
  if (bo >= 4) klaunch(tt_step_mfma<T, 4, BI, LAYOUT>, grid, block, 0, st, tm, a);
  else if (bo == 2) klaunch(tt_step_mfma<T, 2, BI, LAYOUT>, grid, block, 0, st, tm, a);
  else klaunch(tt_step_mfma<T, 1, BI, LAYOUT>, grid, block, 0, st, tm, a);
}

template <typename T, int LAYOUT>
static void launch_mfma(const TTStepArgs<T>& a, hipStream_t st, const LaunchTiming* tm) {
  const int bi = a.b_in <= 1 ? 1 : a.b_in <= 2 ? 2 : a.b_in <= 4 ? 4 : 8;
  const int cap = mfma_bo_cap<T>(bi, LAYOUT);
  const int bo = a.b_out >= cap ? cap : (a.b_out >= 2 ? 2 : 1);
  switch (bi) {
    case 1: launch_mfma_bo<T, LAYOUT, 1>(a, bo, st, tm); break;
    case 2: launch_mfma_bo<T, LAYOUT, 2>(a, bo, st, tm); break;
    case 4: launch_mfma_bo<T, LAYOUT, 4>(a, bo, st, tm); break;
    default: launch_mfma_bo<T, LAYOUT, 8>(a, bo, st, tm); break;
  }
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
  switch (mfma_layout(a)) {
    case TT_ROWS: return launch_mfma<T, TT_ROWS>(a, st, tm);
    case TT_WIDE:
      if constexpr (sizeof(T) == 4) {
        if (a.b_in == 4 && a.b_out == 1) {   // measured: 74 us against 84 for the 16^6 dim 0
          const int steps = a.positions / 64;
          const dim3 grid(steps < 4 * kMaxBlocks ? steps : 4 * kMaxBlocks, (a.b_out + 3) / 4);
          return klaunch(tt_step_shared, grid, dim3(kBlock), 0, st, tm, a);
        }
        return launch_mfma<T, TT_WIDE>(a, st, tm);
      }
      break;
    case TT_INNER: return launch_mfma<T, TT_INNER>(a, st, tm);
    default: break;
  }
  switch (a.mm) {
    case 4: launch_vec_mm<T, 4>(a, st, tm); break;
    case 8: launch_vec_mm<T, 8>(a, st, tm); break;
    default: launch_vec_mm<T, 16>(a, st, tm); break;
  }
}

template <typename T, int E>
static void launch_epi_e(const TTEpiArgs<T>& a, int mode, hipStream_t st, const LaunchTiming* tm) {
  const int64_t nv = a.S / E;
  const int blocks = (nv + kBlock - 1) / kBlock < kMaxBlocks ? static_cast<int>((nv + kBlock - 1) / kBlock)
                                                             : kMaxBlocks;
  const dim3 grid(blocks), block(kBlock);
  switch (mode) {
    case MODE_MAX: klaunch(tt_epilogue<T, MODE_MAX, E>, grid, block, 0, st, tm, a); break;
    case MODE_GREEDY: klaunch(tt_epilogue<T, MODE_GREEDY, E>, grid, block, 0, st, tm, a); break;
    case MODE_EVAL: klaunch(tt_epilogue<T, MODE_EVAL, E>, grid, block, 0, st, tm, a); break;
    default: klaunch(tt_epilogue<T, MODE_RESID, E>, grid, block, 0, st, tm, a); break;
  }
}

template <typename T>
void launch_tt_epilogue(const TTEpiArgs<T>& a, int mode, hipStream_t st, const LaunchTiming* tm) {
  constexpr int W = 16 / static_cast<int>(sizeof(T));
  const uintptr_t ptrs = reinterpret_cast<uintptr_t>(a.V) | reinterpret_cast<uintptr_t>(a.R) |
                         reinterpret_cast<uintptr_t>(a.Vout);
  if (a.S % W == 0 && (ptrs & 15) == 0) launch_epi_e<T, W>(a, mode, st, tm);
  else launch_epi_e<T, 1>(a, mode, st, tm);
}

bool tt_last2_fits(const TTStep2Args& a) {
  const uintptr_t ptrs = reinterpret_cast<uintptr_t>(a.in) | reinterpret_cast<uintptr_t>(a.out);
  return a.S % 256 == 0 && a.b_mid >= 1 && a.b_mid <= 4 && a.b_out >= 1 && a.b_out <= 4 &&
         (ptrs & 15) == 0;
}

void launch_tt_last2(const TTStep2Args& a, hipStream_t st, const LaunchTiming* tm) {
  const int waves = a.S / 256;
  const int blocks = (waves + 3) / 4 < kMaxBlocks ? (waves + 3) / 4 : kMaxBlocks;
  const dim3 grid(blocks), block(kBlock);
  const int bb = a.b_mid <= 1 ? 1 : a.b_mid <= 2 ? 2 : 4;
  const int bo = a.b_out <= 1 ? 1 : a.b_out <= 2 ? 2 : 4;
#define TT2_CASE(B1, B2) \
  if (bb == B1 && bo == B2) return klaunch(tt_step_last2<B1, B2>, grid, block, 0, st, tm, a);
  TT2_CASE(1, 1) TT2_CASE(1, 2) TT2_CASE(1, 4) TT2_CASE(2, 1) TT2_CASE(2, 2) TT2_CASE(2, 4)
  TT2_CASE(4, 1) TT2_CASE(4, 2) TT2_CASE(4, 4)
#undef TT2_CASE
}

template void launch_tt_step<double>(const TTStepArgs<double>&, hipStream_t, const LaunchTiming*);
template void launch_tt_step<float>(const TTStepArgs<float>&, hipStream_t, const LaunchTiming*);
template void launch_tt_epilogue<double>(const TTEpiArgs<double>&, int, hipStream_t,
                                         const LaunchTiming*);
template void launch_tt_epilogue<float>(const TTEpiArgs<float>&, int, hipStream_t,
                                        const LaunchTiming*);

}  // namespace cpm

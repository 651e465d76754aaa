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
// LDS indices are padded by one word per 16 to break bank conflicts of
// strided fibers.
#include <type_traits>

#include "common.cuh"

namespace cpm {

// One pad word per 16: the 16 fibers of a stride-16 block land on distinct
// banks, and for a base B that is a multiple of 16 the padded index splits,
// lpad(B + v) = lpad(B) + lpad(v).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }

// Order the LDS accesses of one wave across the lanes (a wave-local mode
// product reads values that other lanes of the same wave wrote).
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place mode product on an LDS array viewed as [outer][m][inner]:
// X[o, i, in] <- sum_j Tk[i, j] X[o, j, in].  Each thread owns whole fibers
// (o, in), so in-place needs no barrier between its reads and writes.
// WAVE: the calling wave alone works on X (else the whole block).
template <typename T, int MMAX, bool WAVE>
__device__ __forceinline__ void mode_product_lds(const T* Xs, T* X, int outer, int m, int inner,
                                                 FastDiv dv, const T* __restrict__ Tk) {
  const int F = outer * inner;
  const int gid = WAVE ? (threadIdx.x & 63) : threadIdx.x;
  const int gsize = WAVE ? 64 : blockDim.x;
  for (int f = gid; f < F; f += gsize) {
    const int o = static_cast<int>(fdiv(static_cast<uint32_t>(f), dv));
    const int in = f - o * inner;
    const int base = o * m * inner + in;
    T x[MMAX];
#pragma unroll
    for (int j = 0; j < MMAX; ++j)
      if (j < m) x[j] = Xs[lpad(base + j * inner)];
    for (int i = 0; i < m; ++i) {
      const T* Ti = Tk + i * m;
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < MMAX; ++j)
        if (j < m) acc = fma(Ti[j], x[j], acc);
      X[lpad(base + i * inner)] = acc;
    }
  }
  if (WAVE) wave_lds_fence();
  else __syncthreads();
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
typedef double d4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));

// MM_F64: FP64 chains on the FP64 16x16x4 matrix product: operands as the
// FP32 one, but result register r of lane (g, c) holds D[i = g + 4r][fiber c].
// MM_BF16 splits factor and fiber into hi + lo BF16 parts (three products);
// MM_BF16S splits the factor only (two products on the BF16-rounded fiber)
// and keeps the pass-1 intermediate in BF16 as well (see launch_chain).
enum { MM_VALU = 0, MM_F32 = 1, MM_BF16 = 2, MM_F64 = 3, MM_BF16S = 4 };

// The BF16 units share the operand layout of the 16x16x16 product.
constexpr bool bf_unit(int mm) { return mm == MM_BF16 || mm == MM_BF16S; }

template <typename T>
struct AccOf;
template <>
struct AccOf<float> { using type = f4v; };
template <>
struct AccOf<double> { using type = d4v; };

// BF16 bit pattern of x, rounded to nearest even (hardware conversion).
__device__ __forceinline__ uint32_t bf16_bits(float x) {
  return static_cast<uint32_t>(__builtin_bit_cast(uint16_t, static_cast<__bf16>(x)));
}

// BF16 hi + lo split of four FP32 values (hardware round to nearest even).
__device__ __forceinline__ void split_bf16(const float (&x)[4], s4v& hi, s4v& lo) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const __bf16 h = static_cast<__bf16>(x[r]);
    hi[r] = __builtin_bit_cast(short, h);
    lo[r] = __builtin_bit_cast(short, static_cast<__bf16>(x[r] - static_cast<float>(h)));
  }
}

// One 16 x 16 x 16 product: rows k of the B operand held by this lane are
// x[0..3] (fp32 / fp64: k = 4q + g for x[q]; bf16: k = 4g + r for x[r]).
template <typename T, int MM>
__device__ __forceinline__ typename AccOf<T>::type mfma_block(const T (&x)[4], const T (&aw)[4],
                                                              s4v ahi, s4v alo) {
  typename AccOf<T>::type acc = {T(0), T(0), T(0), T(0)};
  if constexpr (MM == MM_F64) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(aw[q], x[q], acc, 0, 0, 0);
  } else if constexpr (MM == MM_F32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aw[q], x[q], acc, 0, 0, 0);
  } else if constexpr (MM == MM_BF16S) {
    // the factor keeps its hi + lo parts (its rounding would be the same
    // for every fiber, a fixed error of the operator); the fiber is rounded
    s4v bhi;
#pragma unroll
    for (int r = 0; r < 4; ++r) bhi[r] = __builtin_bit_cast(short, static_cast<__bf16>(x[r]));
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, acc, 0, 0, 0);
  } else {
    s4v bhi, blo;
    split_bf16(x, bhi, blo);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, acc, 0, 0, 0);
  }
  return acc;
}

template <typename T, int MM, bool WAVE>
__device__ __forceinline__ void mode_product_mfma(const T* Xs, T* X, int outer, int m, int inner,
                                                  FastDiv dv, const T* __restrict__ Tk,
                                                  const uint16_t* __restrict__ Th,
                                                  const uint16_t* __restrict__ Tl) {
  const int lane = threadIdx.x & 63;
  const int wave = WAVE ? 0 : (threadIdx.x >> 6), nw = WAVE ? 1 : (blockDim.x >> 6);
  const int c = lane & 15, g = lane >> 4;
  const int F = outer * inner;
  const int nblk = (F + 15) >> 4;
  T aw[4];
  s4v ahi, alo;
  if (!bf_unit(MM)) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = 4 * q + g;
      aw[q] = (c < m && k < m) ? Tk[c * m + k] : T(0);
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
  // row of the B operand held in x[j] / row of the result in acc[r]
  auto rd_row = [&](int j) { return !bf_unit(MM) ? 4 * j + g : 4 * g + j; };
  auto wr_row = [&](int r) { return MM == MM_F64 ? g + 4 * r : 4 * g + r; };
  auto block_base = [&](int b) {
    const int f = b * 16 + c;
    const int o = static_cast<int>(fdiv(static_cast<uint32_t>(f), dv));
    return o * m * inner + (f - o * inner);
  };
  if (m == 16 && (F & 15) == 0) {
    // full blocks: unguarded loads, two blocks per step so that the LDS
    // reads of both are in flight before the first matrix product
    for (int b0 = wave; b0 < nblk; b0 += 2 * nw) {
      const bool two = b0 + nw < nblk;                 // wave-uniform
      const int base0 = block_base(b0);
      const int base1 = block_base(two ? b0 + nw : b0);
      T x0[4], x1[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        x0[j] = Xs[lpad(base0 + rd_row(j) * inner)];
        x1[j] = Xs[lpad(base1 + rd_row(j) * inner)];
      }
      const auto d0 = mfma_block<T, MM>(x0, aw, ahi, alo);
      const auto d1 = mfma_block<T, MM>(x1, aw, ahi, alo);
#pragma unroll
      for (int r = 0; r < 4; ++r) X[lpad(base0 + wr_row(r) * inner)] = d0[r];
      if (two) {
#pragma unroll
        for (int r = 0; r < 4; ++r) X[lpad(base1 + wr_row(r) * inner)] = d1[r];
      }
    }
  } else {
    for (int b = wave; b < nblk; b += nw) {
      const bool ok = b * 16 + c < F;
      const int base = ok ? block_base(b) : 0;
      T x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = rd_row(j);
        x[j] = (ok && k < m) ? Xs[lpad(base + k * inner)] : T(0);
      }
      const auto d = mfma_block<T, MM>(x, aw, ahi, alo);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr_row(r);
        if (ok && i < m) X[lpad(base + i * inner)] = d[r];
      }
    }
  }
  if (WAVE) wave_lds_fence();
  else __syncthreads();
}

// Matrix-core mode product with m = 16 and an inner stride IN known at
// compile time (IN in {1, 4, 16, 64, 256, 1024}: the pass-1 and pass-2 modes
// of 16^n grids).  The 16 fibers of block b start at B + u with B
// wave-uniform and a multiple of 16, and lpad(B + v) = lpad(B) + lpad(v):
//   IN = 1        : u = 16 c,            lpad(u + k)    = 17 c + k
//   IN % 16 == 0  : u = c,               lpad(u + k IN) = c + k lpad(IN)
//   IN = 4        : u = 64 (c/4) + c%4,  lpad(u + 4 k)  = 68 (c/4) + c%4
//                                                        + 17 (k/4) + 4 (k%4)
// Each row k a lane touches is 4x + y with one of x, y its lane group g
// and the other the register index, so its padded offset is a per-lane part
// plus a compile-time multiple of the register index: one address add per
// block for the four reads and one for the four writes (the rest become LDS
// instruction offsets).
template <typename T, int MM, bool WAVE, int IN>
__device__ __forceinline__ void mode_product_mfma16(const T* Xs, T* X, int outer,
                                                    const T* __restrict__ Tk,
                                                    const uint16_t* __restrict__ Th,
                                                    const uint16_t* __restrict__ Tl) {
  const int lane = threadIdx.x & 63;
  const int wave = WAVE ? 0 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = WAVE ? 1 : (blockDim.x >> 6);
  const int c = lane & 15, g = lane >> 4;
  const int nblk = (outer * IN) >> 4;
  T aw[4];
  s4v ahi, alo;
  if (!bf_unit(MM)) {
#pragma unroll
    for (int q = 0; q < 4; ++q) aw[q] = Tk[c * 16 + 4 * q + g];
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      ahi[r] = static_cast<short>(Th[c * 16 + 4 * g + r]);
      alo[r] = static_cast<short>(Tl[c * 16 + 4 * g + r]);
    }
  }
  // rd_row(j) = 4j + g (FP32, FP64) | 4g + j (BF16);
  // wr_row(r) = g + 4r (FP64)        | 4g + r (FP32, BF16)
  constexpr bool RD_J_HIGH = !bf_unit(MM), WR_R_HIGH = MM == MM_F64;
  constexpr int KS = IN == 1 ? 1 : IN + IN / 16;   // lpad step per row (IN != 4)
  // padded offset of row 4x + y: IN = 4: 17 x + 4 y; else (4 x + y) KS
  constexpr int HI = IN == 4 ? 17 : 4 * KS, LO = IN == 4 ? 4 : KS;
  constexpr int RD_STEP = RD_J_HIGH ? HI : LO, WR_STEP = WR_R_HIGH ? HI : LO;
  const int lu = IN == 1 ? 17 * c : (IN == 4 ? 68 * (c >> 2) + (c & 3) : c);
  const int rd_lane = lu + g * (RD_J_HIGH ? LO : HI);
  const int wr_lane = lu + g * (WR_R_HIGH ? LO : HI);
  auto base_of = [](int b) {
    if (IN == 1) return 256 * b;
    const int o = (16 * b) / IN;
    return o * 16 * IN + (16 * b - o * IN);
  };
  // two blocks per step so that the LDS reads of both are in flight before
  // the first matrix product
  for (int b0 = wave; b0 < nblk; b0 += 2 * nw) {
    const bool two = b0 + nw < nblk;   // wave-uniform
    const int lb0 = lpad(base_of(b0)), lb1 = lpad(base_of(two ? b0 + nw : b0));
    const T* s0 = Xs + lb0 + rd_lane;
    const T* s1 = Xs + lb1 + rd_lane;
    T x0[4], x1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      x0[j] = s0[j * RD_STEP];
      x1[j] = s1[j * RD_STEP];
    }
    const auto d0 = mfma_block<T, MM>(x0, aw, ahi, alo);
    const auto d1 = mfma_block<T, MM>(x1, aw, ahi, alo);
    T* t0 = X + lb0 + wr_lane;
#pragma unroll
    for (int r = 0; r < 4; ++r) t0[r * WR_STEP] = d0[r];
    if (two) {
      T* t1 = X + lb1 + wr_lane;
#pragma unroll
      for (int r = 0; r < 4; ++r) t1[r * WR_STEP] = d1[r];
    }
  }
  if (WAVE) wave_lds_fence();
  else __syncthreads();
}

// Xs: input (may equal X, the output; both viewed as [outer][m][inner]).
template <typename T, int MMAX, int MM, bool WAVE = false>
__device__ __forceinline__ void mode_product(const T* Xs, T* X, int outer, int m, int inner,
                                             FastDiv dv, const T* Tk, const uint16_t* Th,
                                             const uint16_t* Tl) {
  if constexpr (MM == MM_VALU) {
    mode_product_lds<T, MMAX, WAVE>(Xs, X, outer, m, inner, dv, Tk);
  } else {
    if (m == 16 && ((outer * inner) & 15) == 0) {
      if (inner == 1) return mode_product_mfma16<T, MM, WAVE, 1>(Xs, X, outer, Tk, Th, Tl);
      if (inner == 4) return mode_product_mfma16<T, MM, WAVE, 4>(Xs, X, outer, Tk, Th, Tl);
      if (inner == 16) return mode_product_mfma16<T, MM, WAVE, 16>(Xs, X, outer, Tk, Th, Tl);
      if (inner == 64) return mode_product_mfma16<T, MM, WAVE, 64>(Xs, X, outer, Tk, Th, Tl);
      if (inner == 256) return mode_product_mfma16<T, MM, WAVE, 256>(Xs, X, outer, Tk, Th, Tl);
      if (inner == 1024) return mode_product_mfma16<T, MM, WAVE, 1024>(Xs, X, outer, Tk, Th, Tl);
    }
    mode_product_mfma<T, MM, WAVE>(Xs, X, outer, m, inner, dv, Tk, Th, Tl);
  }
}

constexpr int kPass1Block = 256;
constexpr int kPass1RowsBlock = 512;   // at most 8 rows (waves) per block
constexpr int kPass2Block = 1024;
constexpr int kStageRegs = 2;   // staged factor values per thread: n1 * 16^2 <= 2 * 1024

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
    // the first mode product reads the slab vs and writes ws, later ones
    // work in place on ws
    const T* src = vs;
    int outer = 1, inner = C;
    for (int k = a.g.n1; k < n; ++k) {
      const int m = a.g.size[k];
      inner /= m;
      if (a.kinds[t * n + k] != F_IDENT) {
        const int64_t fo = static_cast<int64_t>(t) * a.g.term_stride + a.g.fac_off[k];
        mode_product<T, MMAX, MM>(src, ws, outer, m, inner, a.g.idiv[k], a.fac + fo,
                                  a.facbf + fo, a.facbf_lo + fo);
        src = ws;
      }
      outer *= m;
    }
    T* Wt = a.W + static_cast<int64_t>(t) * a.g.w_term_stride;
    for (int c = threadIdx.x; c < C; c += blockDim.x) {
      const int tile = c >> a.g.ct_shift, clo = c & (a.g.CT - 1);
      Wt[(static_cast<int64_t>(tile) * a.g.Rr + r) * a.g.CT + clo] = src[lpad(c)];
    }
    __syncthreads();
  }
}

// Pass 1, one row per wave (R1 = blockDim / 64 consecutive rows per block).
// Each wave keeps its row of V in registers (PV values per lane) and, per
// term, writes it to its own LDS slab, runs the column-group mode products
// there without block barriers, and then the block writes the R1 slabs out
// as one contiguous run of R1 * CT values per tile of the intermediate
// (whole cache lines, where one row per block writes CT values per tile).
// The column-group factors of the term are staged in LDS for the matrix
// cores.
template <typename T, int MMAX, int MM, int PV>
__global__ __launch_bounds__(kPass1RowsBlock) void chain_pass1_rows(ChainArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  const int C = a.g.C, n = a.g.n, n1 = a.g.n1, Rr = a.g.Rr;
  const int R1 = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int slab = lpad(C) + 1;
  T* base = reinterpret_cast<T*>(smem_raw);
  T* ws = base + w * slab;
  constexpr bool STAGE = (MM != MM_VALU);
  const int cols_off = a.g.fac_off[n1];
  const int cols_len = a.g.term_stride - cols_off;
  T* Fs = base + R1 * slab;
  uint16_t* Fh = reinterpret_cast<uint16_t*>(Fs);
  uint16_t* Fl = Fh + cols_len;
  const int r0 = xcd_block(blockIdx.x, gridDim.x) * R1;
  const int r = r0 + w;
  const bool row_ok = r < Rr;
  const T cs = a.shift_keys ? static_cast<T>(midrange(a.shift_keys)) : T(0);
  T vr[PV];
  {
    const T* Vrow = a.V + static_cast<int64_t>(row_ok ? r : 0) * C;
#pragma unroll
    for (int p = 0; p < PV; ++p) {
      const int c = lane + p * 64;
      vr[p] = (c < C) ? Vrow[c] - cs : T(0);
    }
  }
  const int chunk_shift = a.g.ct_shift + (31 - __builtin_clz(R1));   // log2(R1 * CT)
  const int total = a.g.ntiles << chunk_shift;
  // factors of the next term, loaded before the write-out of the current one
  // (cols_len <= 8 * 16^2 = 4 * kPass1RowsBlock)
  T nf[4];
  uint16_t nh[4], nl[4];
  auto load_fac = [&](int t) {
    if constexpr (STAGE) {
      const int64_t fb = static_cast<int64_t>(t) * a.g.term_stride + cols_off;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = threadIdx.x + j * blockDim.x;
        if (i < cols_len) {
          if (!bf_unit(MM)) {
            nf[j] = a.fac[fb + i];
          } else {
            nh[j] = a.facbf[fb + i];
            nl[j] = a.facbf_lo[fb + i];
          }
        }
      }
    }
  };
  load_fac(0);
  for (int t = 0; t < a.nterms; ++t) {
    if constexpr (STAGE) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int i = threadIdx.x + j * blockDim.x;
        if (i < cols_len) {
          if (!bf_unit(MM)) {
            Fs[i] = nf[j];
          } else {
            Fh[i] = nh[j];
            Fl[i] = nl[j];
          }
        }
      }
    }
    __syncthreads();   // staged factors visible; the slabs of the last term written out
#pragma unroll
    for (int p = 0; p < PV; ++p) {
      const int c = lane + p * 64;
      if (c < C) ws[lpad(c)] = vr[p];
    }
    wave_lds_fence();
    int outer = 1, inner = C;
    for (int k = n1; k < n; ++k) {
      const int m = a.g.size[k];
      inner /= m;
      if (a.kinds[t * n + k] != F_IDENT) {
        if constexpr (STAGE) {
          const int fo = a.g.fac_off[k] - cols_off;
          mode_product<T, MMAX, MM, true>(ws, ws, outer, m, inner, a.g.idiv[k], Fs + fo, Fh + fo,
                                          Fl + fo);
        } else {
          const int64_t fo = static_cast<int64_t>(t) * a.g.term_stride + a.g.fac_off[k];
          mode_product<T, MMAX, MM, true>(ws, ws, outer, m, inner, a.g.idiv[k], a.fac + fo,
                                          a.facbf + fo, a.facbf_lo + fo);
        }
      }
      outer *= m;
    }
    __syncthreads();   // all slabs of this term complete
    if (t + 1 < a.nterms) load_fac(t + 1);
    // W_t[tile][r0 .. r0 + R1)[0 .. CT): q runs over whole chunks of R1 * CT
    T* Wt = a.W + static_cast<int64_t>(t) * a.g.w_term_stride;
    constexpr int VW = 16 / sizeof(T), LOG_VW = sizeof(T) == 4 ? 2 : 1;
    if constexpr (MM == MM_BF16S) {
      // BF16 intermediate: units of 8 consecutive values of one chunk (R1
      // rows x CT columns of a tile), rounded to nearest even, one 16-byte
      // store each (the host guarantees whole chunks of a multiple of 8
      // values, every row of the block in range and whole tiles)
      uint16_t* Wb = reinterpret_cast<uint16_t*>(a.W) + static_cast<int64_t>(t) * a.g.w_term_stride;
      const int ushift = chunk_shift - 3;
      for (int qv = threadIdx.x; qv < (total >> 3); qv += blockDim.x) {
        const int tile = qv >> ushift;
        const int rem = (qv & ((1 << ushift) - 1)) << 3;
        uint32_t pk[4];
#pragma unroll
        for (int e = 0; e < 8; e += 2) {
          const int q0 = rem + e, q1 = rem + e + 1;
          const T v0 = base[(q0 >> a.g.ct_shift) * slab + lpad(tile * a.g.CT + (q0 & (a.g.CT - 1)))];
          const T v1 = base[(q1 >> a.g.ct_shift) * slab + lpad(tile * a.g.CT + (q1 & (a.g.CT - 1)))];
          pk[e >> 1] = bf16_bits(static_cast<float>(v0)) | (bf16_bits(static_cast<float>(v1)) << 16);
        }
        *reinterpret_cast<uint4*>(Wb + (static_cast<int64_t>(tile) * Rr + r0) * a.g.CT + rem) =
            make_uint4(pk[0], pk[1], pk[2], pk[3]);
      }
    } else if (a.g.CT >= VW && C % a.g.CT == 0) {
      // 16-byte units: VW consecutive columns of one row of one tile, one
      // vector store (the units never cross a tile, and with one pad word per
      // 16 never a pad word in LDS)
      using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
      const int vshift = chunk_shift - LOG_VW;
      for (int qv = threadIdx.x; qv < (total >> LOG_VW); qv += blockDim.x) {
        const int tile = qv >> vshift;
        const int rem = (qv & ((1 << vshift) - 1)) << LOG_VW;
        const int i = rem >> a.g.ct_shift;
        if (r0 + i < Rr) {
          const T* src = base + i * slab + lpad(tile * a.g.CT + (rem & (a.g.CT - 1)));
          V v;
          T* pv = reinterpret_cast<T*>(&v);
#pragma unroll
          for (int e = 0; e < VW; ++e) pv[e] = src[e];
          *reinterpret_cast<V*>(Wt + (static_cast<int64_t>(tile) * Rr + r0) * a.g.CT + rem) = v;
        }
      }
    } else {
      for (int q = threadIdx.x; q < total; q += blockDim.x) {
        const int tile = q >> chunk_shift;
        const int rem = q & ((1 << chunk_shift) - 1);
        const int i = rem >> a.g.ct_shift, clo = rem & (a.g.CT - 1);
        const int c = tile * a.g.CT + clo;
        if (r0 + i < Rr && c < C)
          Wt[(static_cast<int64_t>(tile) * Rr + r0) * a.g.CT + rem] = base[i * slab + lpad(c)];
      }
    }
  }
}

// EPT consecutive values from p (16-byte aligned) into registers.
template <typename T, int EPT>
__device__ __forceinline__ void load_run(const T* __restrict__ p, T (&d)[EPT]) {
  constexpr int VW = 16 / sizeof(T);
  if constexpr (EPT % VW == 0) {
    using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
#pragma unroll
    for (int q = 0; q < EPT / VW; ++q) {
      const V v = reinterpret_cast<const V*>(p)[q];
      const T* pv = reinterpret_cast<const T*>(&v);
#pragma unroll
      for (int i = 0; i < VW; ++i) d[q * VW + i] = pv[i];
    }
  } else {
#pragma unroll
    for (int j = 0; j < EPT; ++j) d[j] = p[j];
  }
}

// EPT consecutive BF16 values from p (aligned to 2 EPT bytes, at most 16)
// widened to FP32.
template <int EPT>
__device__ __forceinline__ void load_run_bf16(const uint16_t* __restrict__ p, float (&d)[EPT]) {
  auto put = [&](int j, uint32_t w) {
    d[j] = __uint_as_float(w << 16);
    d[j + 1] = __uint_as_float(w & 0xFFFF0000u);
  };
  if constexpr (EPT % 8 == 0) {
#pragma unroll
    for (int q = 0; q < EPT / 8; ++q) {
      const uint4 v = reinterpret_cast<const uint4*>(p)[q];
      put(8 * q, v.x);
      put(8 * q + 2, v.y);
      put(8 * q + 4, v.z);
      put(8 * q + 6, v.w);
    }
  } else if constexpr (EPT == 4) {
    const uint2 v = *reinterpret_cast<const uint2*>(p);
    put(0, v.x);
    put(2, v.y);
  } else {
    static_assert(EPT == 2, "EPT of a BF16 run: 2, 4 or a multiple of 8");
    put(0, *reinterpret_cast<const uint32_t*>(p));
  }
}

// Thread i owns the EPT consecutive tile elements e0 = i * EPT ...; EPT
// divides 32, so their padded LDS indices are lpad(e0) + j.
template <typename T, int MMAX, int MODE, int EPT, int MM>
__global__ __launch_bounds__(kPass2Block) void chain_pass2(ChainArgs<T> a) {
  static_assert(32 % EPT == 0, "EPT must divide 32");
  extern __shared__ unsigned char smem_raw[];
  T* X = reinterpret_cast<T*>(smem_raw);
  __shared__ int act_used[kMaxActions + 1];
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int CT = a.g.CT, C = a.g.C, n1 = a.g.n1, n = a.g.n;
  const int TE = a.g.Rr * CT;
  const int e0 = threadIdx.x * EPT;
  T* Xe = X + lpad(e0);
  const bool full = e0 + EPT <= TE;                   // all EPT elements in the tile
  // Matrix-core units read the row-group factors of the current term from
  // LDS; they are fetched with the next tile, so no global load of the mode
  // products waits behind the tile prefetch.
  constexpr bool STAGE = (MM != MM_VALU);
  const int rows_len = (n1 < n) ? a.g.fac_off[n1] : a.g.term_stride;
  T* Fs = X + lpad(TE) + 1;
  uint16_t* Fh = reinterpret_cast<uint16_t*>(Fs);
  uint16_t* Fl = Fh + rows_len;
  T nf[kStageRegs];
  uint16_t nh[kStageRegs], nl[kStageRegs];

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
      const int s = state_of(e0 + j, v);
      if (v) {
        pold[j] = a.pi_in[s];
        if (MODE == MODE_EVAL || MODE == MODE_RESID) act_used[pold[j]] = 1;
      }
    }
  }
  if (MODE == MODE_EVAL || MODE == MODE_RESID) __syncthreads();

  // Terms are visited action by action; the tile of the next term is loaded
  // into registers while the current one is in the mode products, so the
  // global loads overlap the LDS / matrix-core work.
  const int64_t tile_off = static_cast<int64_t>(tile) * TE;
  const bool vec_ok = (TE % (16 / sizeof(T)) == 0) &&
                      (reinterpret_cast<uintptr_t>(a.W) % 16 == 0) &&
                      ((a.g.w_term_stride * sizeof(T)) % 16 == 0);
  const bool skip_unused = (MODE == MODE_EVAL || MODE == MODE_RESID);
  auto used_from = [&](int act) {
    while (skip_unused && act < a.A && !act_used[act]) ++act;
    return act;
  };
  T nx[EPT];
  auto load_tile = [&](int t) {
    if constexpr (MM == MM_BF16S) {
      // BF16 intermediate (pass 1 of the same unit wrote it)
      const uint16_t* Wb = reinterpret_cast<const uint16_t*>(a.W) +
                           static_cast<int64_t>(t) * a.g.w_term_stride + tile_off + e0;
      if (full) {
        float f[EPT];
        load_run_bf16<EPT>(Wb, f);
#pragma unroll
        for (int j = 0; j < EPT; ++j) nx[j] = static_cast<T>(f[j]);
      } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j)
          nx[j] = (e0 + j < TE) ? static_cast<T>(__uint_as_float(static_cast<uint32_t>(Wb[j]) << 16))
                                : T(0);
      }
    } else {
      const T* Wt = a.W + static_cast<int64_t>(t) * a.g.w_term_stride + tile_off + e0;
      if (full && vec_ok) {
        load_run<T, EPT>(Wt, nx);
      } else {
#pragma unroll
        for (int j = 0; j < EPT; ++j) nx[j] = (e0 + j < TE) ? Wt[j] : T(0);
      }
    }
  };
  auto load_fac = [&](int t) {
    if constexpr (STAGE) {
      const int64_t base = static_cast<int64_t>(t) * a.g.term_stride;
#pragma unroll
      for (int i = 0; i < kStageRegs; ++i) {
        const int idx = threadIdx.x + i * kPass2Block;
        if (idx < rows_len) {
          if (!bf_unit(MM)) {
            nf[i] = a.fac[base + idx];
          } else {
            nh[i] = a.facbf[base + idx];
            nl[i] = a.facbf_lo[base + idx];
          }
        }
      }
    }
  };
  int act = used_from(0);
  int t = act < a.A ? a.term_start[act] : 0;
  if (act < a.A) {
    load_fac(t);
    load_tile(t);
  }
  while (act < a.A) {
    if constexpr (STAGE) {
#pragma unroll
      for (int i = 0; i < kStageRegs; ++i) {
        const int idx = threadIdx.x + i * kPass2Block;
        if (idx < rows_len) {
          if (!bf_unit(MM)) {
            Fs[idx] = nf[i];
          } else {
            Fh[idx] = nh[i];
            Fl[idx] = nl[i];
          }
        }
      }
    }
    if (full) {
#pragma unroll
      for (int j = 0; j < EPT; ++j) Xe[j] = nx[j] - cs_in;
    } else {
#pragma unroll
      for (int j = 0; j < EPT; ++j)
        if (e0 + j < TE) Xe[j] = nx[j] - cs_in;
    }
    const bool last_of_act = (t + 1 == a.term_start[act + 1]);
    const int act2 = last_of_act ? used_from(act + 1) : act;
    const int t2 = last_of_act ? (act2 < a.A ? a.term_start[act2] : 0) : t + 1;
    if (act2 < a.A) {
      load_fac(t2);
      load_tile(t2);
    }
    __syncthreads();
    int outer = 1, inner = TE;
    for (int k = 0; k < n1; ++k) {
      const int m = a.g.size[k];
      inner /= m;
      if (a.kinds[t * n + k] != F_IDENT) {
        if constexpr (STAGE) {
          const int fo = a.g.fac_off[k];
          mode_product<T, MMAX, MM>(X, X, outer, m, inner, a.g.idiv[k], Fs + fo, Fh + fo, Fl + fo);
        } else {
          const int64_t fo = static_cast<int64_t>(t) * a.g.term_stride + a.g.fac_off[k];
          mode_product<T, MMAX, MM>(X, X, outer, m, inner, a.g.idiv[k], a.fac + fo,
                                    a.facbf + fo, a.facbf_lo + fo);
        }
      }
      outer *= m;
    }
    const T lam = a.lam[t];
    if (full) {
      T x[EPT];
#pragma unroll
      for (int j = 0; j < EPT; ++j) x[j] = Xe[j];
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        if (MODE == MODE_EVAL || MODE == MODE_RESID) {
          acc[j] = (pold[j] == act) ? fma(lam, x[j], acc[j]) : acc[j];
        } else {
          acc[j] = fma(lam, x[j], acc[j]);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        if (e0 + j < TE) {
          const T x = Xe[j];
          if (MODE == MODE_EVAL || MODE == MODE_RESID) {
            if (pold[j] == act) acc[j] = fma(lam, x, acc[j]);
          } else {
            acc[j] = fma(lam, x, acc[j]);
          }
        }
      }
    }
    __syncthreads();
    if (last_of_act) {
      if (MODE == MODE_MAX) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          best[j] = acc[j] > best[j] ? acc[j] : best[j];
          acc[j] = T(0);
        }
      } else if (MODE == MODE_GREEDY) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
          bool v;
          const int s = state_of(e0 + j, v);
          if (v) {
            const T g = is_terminal(a.term_bits, s) ? T(0) : a.gamma;
            const T q = fma(g, acc[j] + cs, a.R[s]);
            tie_update(q, act, tol, best[j], bi[j]);
            if (act == pold[j]) qold[j] = q;
          }
          acc[j] = T(0);
        }
      }
    }
    act = act2;
    t = t2;
  }

  double res = 0.0;
  unsigned changed = 0;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    bool v;
    const int s = state_of(e0 + j, v);
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
static void launch_pass1_m(const ChainArgs<T>& a, hipStream_t st, const LaunchTiming* tm) {
  if (a.g.r1 > 0) {
    const int R1 = a.g.r1;
    const int cols_len = a.g.term_stride - a.g.fac_off[a.g.n1];
    const size_t sh = sizeof(T) * static_cast<size_t>(R1) * (a.g.C + (a.g.C >> 4) + 1) +
                      (MM != MM_VALU ? sizeof(T) * static_cast<size_t>(cols_len) : 0);
    const dim3 grid((a.g.Rr + R1 - 1) / R1), block(64 * R1);
    const int pv = (a.g.C + 63) / 64;
    if (pv <= 16) klaunch(chain_pass1_rows<T, MMAX, MM, 16>, grid, block, sh, st, tm, a);
    else if (pv <= 32) klaunch(chain_pass1_rows<T, MMAX, MM, 32>, grid, block, sh, st, tm, a);
    else klaunch(chain_pass1_rows<T, MMAX, MM, 64>, grid, block, sh, st, tm, a);
    return;
  }
  const size_t sh = sizeof(T) * (2 * (static_cast<size_t>(a.g.C) + (a.g.C >> 4) + 1) + 2);
  klaunch(chain_pass1<T, MMAX, MM>, dim3(a.g.Rr), dim3(kPass1Block), sh, st, tm, a);
}

template <typename T, int MMAX, int MODE, int MM>
static void launch_pass2_mm(const ChainArgs<T>& a, hipStream_t st, const LaunchTiming* tm) {
  const int TE = a.g.Rr * a.g.CT;
  const int ept = (TE + kPass2Block - 1) / kPass2Block;
  const int rows_len = (a.g.n1 < a.g.n) ? a.g.fac_off[a.g.n1] : a.g.term_stride;
  const size_t sh = sizeof(T) * (static_cast<size_t>(TE) + (TE >> 4) + 2) +
                    (MM != MM_VALU ? sizeof(T) * static_cast<size_t>(rows_len) : 0);
  const dim3 grid(a.g.ntiles), block(kPass2Block);
  if (ept <= 2) klaunch(chain_pass2<T, MMAX, MODE, 2, MM>, grid, block, sh, st, tm, a);
  else if (ept <= 4) klaunch(chain_pass2<T, MMAX, MODE, 4, MM>, grid, block, sh, st, tm, a);
  else if (ept <= 8) klaunch(chain_pass2<T, MMAX, MODE, 8, MM>, grid, block, sh, st, tm, a);
  else klaunch(chain_pass2<T, MMAX, MODE, 16, MM>, grid, block, sh, st, tm, a);
}

template <typename T, int MMAX, int MM>
static void launch_pass2_m(const ChainArgs<T>& a, int mode, hipStream_t st,
                           const LaunchTiming* tm) {
  switch (mode) {
    case MODE_MAX: launch_pass2_mm<T, MMAX, MODE_MAX, MM>(a, st, tm); break;
    case MODE_GREEDY: launch_pass2_mm<T, MMAX, MODE_GREEDY, MM>(a, st, tm); break;
    case MODE_EVAL: launch_pass2_mm<T, MMAX, MODE_EVAL, MM>(a, st, tm); break;
    default: launch_pass2_mm<T, MMAX, MODE_RESID, MM>(a, st, tm); break;
  }
}

// Unit of one group's mode products: matrix cores when every mode of the
// group has m_k <= 16 (FP32 from 5 up, BF16 always), vector ALUs otherwise.
static int pick_unit(int mmax, int unit) {
  if (unit == CHAIN_BF16) return mmax <= 16 ? MM_BF16 : MM_VALU;
  if (unit == CHAIN_F32_MFMA) return (mmax > 4 && mmax <= 16) ? MM_F32 : MM_VALU;
  if (unit == CHAIN_F64_MFMA) return (mmax > 4 && mmax <= 16) ? MM_F64 : MM_VALU;
  return MM_VALU;
}

template <typename T>
static void launch_pass1(const ChainArgs<T>& a, int mm, hipStream_t st, const LaunchTiming* tm) {
  if constexpr (std::is_same<T, float>::value) {
    if (mm == MM_F32) return launch_pass1_m<T, 16, MM_F32>(a, st, tm);
    if (mm == MM_BF16) return launch_pass1_m<T, 16, MM_BF16>(a, st, tm);
    if (mm == MM_BF16S) return launch_pass1_m<T, 16, MM_BF16S>(a, st, tm);
  } else {
    if (mm == MM_F64) return launch_pass1_m<T, 16, MM_F64>(a, st, tm);
  }
  switch (pick_mmax(a.g.mmax_col)) {
    case 4: return launch_pass1_m<T, 4, MM_VALU>(a, st, tm);
    case 16: return launch_pass1_m<T, 16, MM_VALU>(a, st, tm);
    default: return launch_pass1_m<T, 32, MM_VALU>(a, st, tm);
  }
}

template <typename T>
static void launch_pass2(const ChainArgs<T>& a, int mode, int mm, hipStream_t st,
                         const LaunchTiming* tm) {
  if constexpr (std::is_same<T, float>::value) {
    if (mm == MM_F32) return launch_pass2_m<T, 16, MM_F32>(a, mode, st, tm);
    if (mm == MM_BF16) return launch_pass2_m<T, 16, MM_BF16>(a, mode, st, tm);
    if (mm == MM_BF16S) return launch_pass2_m<T, 16, MM_BF16S>(a, mode, st, tm);
  } else {
    if (mm == MM_F64) return launch_pass2_m<T, 16, MM_F64>(a, mode, st, tm);
  }
  switch (pick_mmax(a.g.mmax_row)) {
    case 4: return launch_pass2_m<T, 4, MM_VALU>(a, mode, st, tm);
    case 16: return launch_pass2_m<T, 16, MM_VALU>(a, mode, st, tm);
    default: return launch_pass2_m<T, 32, MM_VALU>(a, mode, st, tm);
  }
}

// The single-product BF16 unit (one BF16 product per block, intermediate in
// BF16) runs when both passes exist and every mode has 8 to 16 states (the
// relative rounding of the smaller factors' few entries would reach the BF16
// tolerance; they keep the hi + lo split and an FP32 intermediate), and when
// pass 1 writes whole 16-byte units: one row per wave, every row of every
// block in range, whole tiles, 8 | R1 CT.
static bool bf16_single_ok(const ChainGeom& g) {
  if (g.n1 >= g.n || g.r1 <= 0) return false;
  for (int k = 0; k < g.n; ++k)
    if (g.size[k] < 8 || g.size[k] > 16) return false;
  return g.Rr % g.r1 == 0 && g.C % g.CT == 0 && (g.r1 * g.CT) % 8 == 0 &&
         (static_cast<int64_t>(g.Rr) * g.CT) % 8 == 0;
}

// tm: start recorded at the first pass, stop after the second.
template <typename T>
void launch_chain(const ChainArgs<T>& a, int mode, int unit, hipStream_t st,
                  const LaunchTiming* tm) {
  if constexpr (std::is_same<T, float>::value) {
    // BF16 and FP32 max sweeps of 16^6 grids: every mode product in registers
    if (mode == MODE_MAX && chain16_bf16_ok(a.g)) {
      if (unit == CHAIN_BF16) return launch_chain16_bf16(a, st, tm);
      if (unit == CHAIN_F32_MFMA) return launch_chain16_f32(a, st, tm);
    }
  }
  const bool two = a.g.n1 < a.g.n;
  const LaunchTiming t1{tm ? tm->start : nullptr, nullptr};
  const LaunchTiming t2{two ? nullptr : (tm ? tm->start : nullptr), tm ? tm->stop : nullptr};
  int mm1 = pick_unit(a.g.mmax_col, unit), mm2 = pick_unit(a.g.mmax_row, unit);
  if (std::is_same<T, float>::value && unit == CHAIN_BF16 && bf16_single_ok(a.g))
    mm1 = mm2 = MM_BF16S;
  if (two) launch_pass1(a, mm1, st, tm ? &t1 : nullptr);
  launch_pass2(a, mode, mm2, st, tm ? &t2 : nullptr);
}

template void launch_chain<double>(const ChainArgs<double>&, int, int, hipStream_t,
                                   const LaunchTiming*);
template void launch_chain<float>(const ChainArgs<float>&, int, int, hipStream_t,
                                  const LaunchTiming*);

}  // namespace cpm

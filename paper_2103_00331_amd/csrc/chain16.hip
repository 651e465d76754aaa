// K2, register-resident BF16 and FP32 units for grids of six modes of 16
// states (both groups three modes of 16, so one row of pass 1 and one column
// of pass 2 is a 16 x 16 x 16 tensor of 4096 values).  The BF16 unit is
// described here; the FP32 unit, further down, follows it with the FP32
// matrix product.
//
// The operator is the one of the two-pass chain: pass 1 applies the column
// group's factors of every term to each row of V (minus the midrange shift),
// pass 2 the row group's factors to each column of the intermediate, scales
// by the term weight, sums the terms of an action and takes the max over
// actions, then forms Eq. 1's V' and the sup-norm residual (the CP form of
// Sec. 2.2 applied without forming P_a).  The BF16 rounding points are those
// of the single-product BF16 unit: each mode product rounds its input fiber
// to BF16 once and multiplies it by the factor in hi + lo parts with FP32
// accumulation; the intermediate is held in BF16.
//
// Instead of running each mode product through LDS with a barrier between
// modes, a wave keeps its whole 16^3 tensor in registers (64 BF16 values per
// lane, packed in pairs) and chains the matrix products directly.  With the
// 16 x 16 x 16 BF16 product (lane l = 16 g + c holds A[c][4g..4g+3],
// B[4g..4g+3][c] and returns D[4g..4g+3][c]), a block X[p][q] held as
// "lane (g, c), register i = X[4g + i][c]" is both a valid A operand (as
// X^T) and a valid B operand:
//   A form  D = X^T F^T : contracts p, result block (q, new index);
//   B form  D = F X     : contracts p, result block (new index, q);
// the factor registers (F[c][4g..4g+3]) are the same in both.  Two A-form
// products contract the two in-block indices; the third index is the block
// number (16 blocks per lane), which a 4 x 4 exchange of lane groups against
// block numbers (v_permlane32_swap / v_permlane16_swap, plus a swap of BF16
// halves) moves into the block's row, where the last product contracts it.
//
//   pass 1 (8 rows per block, one per wave): row r's tensor Z[x3][x4][x5]
//     starts as blocks b = x3, X[p = x4][q = x5]; A(T4), A(T5), exchange,
//     A(T3) leave y[y3][y4][y5] with y3 = c, y4 = b, y5 = 4g + i: four
//     consecutive columns per lane and block, stored to the wave's LDS row
//     (8-byte stores, padded by 8 values per 256 so the 64 lanes hit distinct
//     banks); the block then writes the intermediate tile by tile, 8 rows x
//     8 columns = one 128-byte line per tile: layout [term][tile][row][8].
//     (Tiles of 4 columns would need 16 rows per block for whole lines, and
//     a 16-row block fills a CU's LDS alone; half-line writes measured worse.)
//   pass 2 (half a tile, 4 columns, per block, one column per wave; two blocks
//     per CU, so one computes while the other waits for its next tile; the
//     two halves of a tile are neighbouring blocks on one XCD and share its
//     lines in L2): the 8-byte halves of the tile's rows are copied into 4 LDS
//     column arrays (padded as above); column cc's tensor
//     X[x0][x1][x2] is read as blocks b = x1, X[p = x2][q = x0] (four
//     consecutive rows per 8-byte LDS read); A(T2), A(T0), exchange, then
//     B(lambda T1) accumulates straight into the action's FP32 sum (the
//     matrix product's accumulator input), which leaves y0 = c, y1 = 4g + i,
//     y2 = b.
#include "common.cuh"

namespace cpm {

namespace {

typedef short s4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));

constexpr int kFib = 4096;      // values of one row (pass 1) / one column (pass 2)
constexpr int kP1Rows = 8;      // pass 1: rows per block, one per wave
constexpr int kTile = 8;        // columns per tile of the intermediate
constexpr int kP2Cols = 4;      // pass 2: columns per block (half a tile), one per wave
// LDS arrays: 4096 values + 8 per 256 (pad16); the pass-1 rows get 16 more
// (a row stride of 8 words mod 64 banks) so that the 8 rows x 2 tiles of a
// 16-byte read by 16 lanes fall on distinct banks.
constexpr int kColArr = kFib + 16 * 8;    // 4224
constexpr int kSlab = kColArr + 16;       // 4240

__device__ __forceinline__ int pad16(int v) { return v + ((v >> 8) << 3); }

// Two FP32 values as a packed BF16 pair (round to nearest even), a low.
__device__ __forceinline__ uint32_t pk(float a, float b) {
  const bf2v p = {static_cast<__bf16>(a), static_cast<__bf16>(b)};
  return __builtin_bit_cast(uint32_t, p);
}

__device__ __forceinline__ s4v op(uint32_t lo, uint32_t hi) {
  const u2v v = {lo, hi};
  return __builtin_bit_cast(s4v, v);
}

__device__ __forceinline__ f4v mfma(s4v a, s4v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Factor registers of mode k of term t: F[c][4g .. 4g + 3] as BF16 hi and lo.
struct Fac16 {
  s4v hi, lo;
};

__device__ __forceinline__ Fac16 fac16(const ChainArgs<float>& a, int t, int k, int lane) {
  const int64_t o = static_cast<int64_t>(t) * a.g.term_stride + a.g.fac_off[k] + (lane & 15) * 16 +
                    4 * (lane >> 4);
  Fac16 f;
  f.hi = *reinterpret_cast<const s4v*>(a.facbf + o);
  f.lo = *reinterpret_cast<const s4v*>(a.facbf_lo + o);
  return f;
}

// The FP32 factor values F[c][4g .. 4g + 3] of mode k of term t.
__device__ __forceinline__ float4 fac32(const ChainArgs<float>& a, int t, int k, int lane) {
  const int64_t o = static_cast<int64_t>(t) * a.g.term_stride + a.g.fac_off[k] + (lane & 15) * 16 +
                    4 * (lane >> 4);
  return *reinterpret_cast<const float4*>(a.fac + o);
}

// lambda times the FP32 factor values v, split into BF16 hi + lo.
__device__ __forceinline__ Fac16 split_scaled(float4 v, float lam) {
  const float x[4] = {lam * v.x, lam * v.y, lam * v.z, lam * v.w};
  Fac16 f;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const __bf16 h = static_cast<__bf16>(x[r]);
    f.hi[r] = __builtin_bit_cast(short, h);
    f.lo[r] = __builtin_bit_cast(short, static_cast<__bf16>(x[r] - static_cast<float>(h)));
  }
  return f;
}

// One A-form product per block: u[b] <- BF16(X_b^T F^T) in place.
__device__ __forceinline__ void aform16(uint32_t (&u)[16][2], const Fac16& f) {
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    const s4v x = op(u[b][0], u[b][1]);
    f4v d = {0.f, 0.f, 0.f, 0.f};
    d = mfma(x, f.lo, d);
    d = mfma(x, f.hi, d);
    u[b][0] = pk(d[0], d[1]);
    u[b][1] = pk(d[2], d[3]);
  }
}

// u[b][h] holds X[b][p][c] for p = 4g + 2h + e (BF16 half e).  Afterwards it
// holds X'[b][p][c] = X[p][b][c]: block number and block row trade places.
// (a) for each (b mod 4, h), the four registers b = 4m + b mod 4 are
//     transposed against the four lane groups (32-lane, then 16-lane swaps);
// (b) BF16 halves are exchanged between register pairs.
__device__ __forceinline__ void exchange16(uint32_t (&u)[16][2]) {
  uint32_t R[4][2][4];
#pragma unroll
  for (int bl = 0; bl < 4; ++bl) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      uint32_t x0 = u[bl][h], x1 = u[4 + bl][h], x2 = u[8 + bl][h], x3 = u[12 + bl][h];
      auto s02 = __builtin_amdgcn_permlane32_swap(x0, x2, false, false);
      auto s13 = __builtin_amdgcn_permlane32_swap(x1, x3, false, false);
      auto s01 = __builtin_amdgcn_permlane16_swap(s02[0], s13[0], false, false);
      auto s23 = __builtin_amdgcn_permlane16_swap(s02[1], s13[1], false, false);
      R[bl][h][0] = s01[0];
      R[bl][h][1] = s01[1];
      R[bl][h][2] = s23[0];
      R[bl][h][3] = s23[1];
    }
  }
#pragma unroll
  for (int bh = 0; bh < 4; ++bh) {
#pragma unroll
    for (int bm = 0; bm < 2; ++bm) {
#pragma unroll
      for (int H = 0; H < 2; ++H) {
        const uint32_t lo = R[2 * H][bm][bh], hi = R[2 * H + 1][bm][bh];
        u[4 * bh + 2 * bm][H] = (lo & 0xFFFFu) | (hi << 16);
        u[4 * bh + 2 * bm + 1][H] = (lo >> 16) | (hi & 0xFFFF0000u);
      }
    }
  }
}

__global__ __launch_bounds__(kP1Rows * 64) void chain16_pass1(ChainArgs<float> a) {
  __shared__ __align__(16) uint16_t slab[kP1Rows * kSlab];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int r0 = xcd_block(blockIdx.x, gridDim.x) * kP1Rows;
  const float cs = a.shift_keys ? midrange(a.shift_keys) : 0.f;
  // row r0 + w of V - cs, blocks b = x3 with X[p = x4][q = x5]: lane (g, c)
  // register (b, i) holds offset 256 b + 16 (4 g + i) + c
  uint32_t v[16][2];
  {
    const float* Vr = a.V + static_cast<int64_t>(r0 + w) * kFib + 64 * g + c;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
        v[b][h] = pk(Vr[256 * b + 32 * h] - cs, Vr[256 * b + 32 * h + 16] - cs);
    }
  }
  uint16_t* my = slab + w * kSlab + pad16(256 * c + 4 * g);
  uint16_t* Wb = reinterpret_cast<uint16_t*>(a.W);
  const int64_t S = a.g.S, Rr = a.g.Rr;
  // The next term's factors are loaded just before this term's stores: loads
  // and stores retire in order, so waiting for the factors never waits for
  // the stores (the scheduling barriers keep that order).
  Fac16 f3 = fac16(a, 0, 3, lane), f4 = fac16(a, 0, 4, lane), f5 = fac16(a, 0, 5, lane);
  for (int t = 0; t < a.nterms; ++t) {
    uint32_t u[16][2];
#pragma unroll
    for (int b = 0; b < 16; ++b) {     // A(T4): (p = x5, q = y4)
      const s4v x = op(v[b][0], v[b][1]);
      f4v d = {0.f, 0.f, 0.f, 0.f};
      d = mfma(x, f4.lo, d);
      d = mfma(x, f4.hi, d);
      u[b][0] = pk(d[0], d[1]);
      u[b][1] = pk(d[2], d[3]);
    }
    aform16(u, f5);                    // (p = y4, q = y5)
    exchange16(u);                     // blocks y4, (p = x3, q = y5)
#pragma unroll
    for (int b = 0; b < 16; ++b) {     // A(T3): (p = y5, q = y3); column 256 c + 16 b + 4 g + i
      const s4v x = op(u[b][0], u[b][1]);
      f4v d = {0.f, 0.f, 0.f, 0.f};
      d = mfma(x, f3.lo, d);
      d = mfma(x, f3.hi, d);
      const u2v p = {pk(d[0], d[1]), pk(d[2], d[3])};
      *reinterpret_cast<u2v*>(my + 16 * b) = p;
    }
    __syncthreads();
    {
      const int tn = min(t + 1, a.nterms - 1);
      f3 = fac16(a, tn, 3, lane);
      f4 = fac16(a, tn, 4, lane);
      f5 = fac16(a, tn, 5, lane);
    }
    __builtin_amdgcn_sched_barrier(0);
    // the block's rows, tile by tile: unit q = (tile, row), 16 bytes each
    uint16_t* Wt = Wb + static_cast<int64_t>(t) * S;
    constexpr int kUnits = (kFib / kTile) * kP1Rows;   // 16-byte units of the block
#pragma unroll
    for (int j = 0; j < kUnits / (kP1Rows * 64); ++j) {
      const int q = threadIdx.x + j * (kP1Rows * 64);
      const int tl = q / kP1Rows, ww = q % kP1Rows;
      const uint4 val = *reinterpret_cast<const uint4*>(slab + ww * kSlab + pad16(kTile * tl));
      *reinterpret_cast<uint4*>(Wt + (static_cast<int64_t>(tl) * Rr + r0 + ww) * kTile) = val;
    }
    __syncthreads();
  }
}

// two waves per SIMD: two blocks of four waves per CU
__global__ __launch_bounds__(kP2Cols * 64, 2) void chain16_pass2(ChainArgs<float> a) {
  __shared__ __align__(16) uint16_t cols[kP2Cols * kColArr];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int tile = blk >> 1, half = blk & 1;
  const int64_t S = a.g.S;
  const uint16_t* Wb = reinterpret_cast<const uint16_t*>(a.W) + static_cast<int64_t>(tile) * kFib * kTile +
                       threadIdx.x * 2 * kTile + half * kP2Cols;
  // this block's halves of rows 2u and 2u + 1 of the tile, u = j * 256 + thread
  constexpr int kLoads = kFib / 2 / (kP2Cols * 64);
  uint4 nx[kLoads];
  auto load = [&](int t) {
    const uint16_t* p = Wb + static_cast<int64_t>(t) * S;
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      const u2v r0h = *reinterpret_cast<const u2v*>(p + j * (kP2Cols * 64) * 2 * kTile);
      const u2v r1h = *reinterpret_cast<const u2v*>(p + j * (kP2Cols * 64) * 2 * kTile + kTile);
      nx[j] = make_uint4(r0h[0], r0h[1], r1h[0], r1h[1]);
    }
  };
  f4v acc[16], best[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    acc[b] = f4v{0.f, 0.f, 0.f, 0.f};
    best[b] = f4v{-INFINITY, -INFINITY, -INFINITY, -INFINITY};
  }
  const float cs = a.shift_keys ? midrange(a.shift_keys) : 0.f;
  const uint16_t* mc = cols + w * kColArr + pad16(256 * c + 4 * g);
  int act = 0;
  if (a.nterms > 0) load(0);
  for (int t = 0; t < a.nterms; ++t) {
    __syncthreads();   // the previous term's column reads are done
#pragma unroll
    for (int j = 0; j < kLoads; ++j) {
      // rows 2u (words x, y) and 2u + 1 (words z, w), columns 0..3; column e
      // gets the pair (row 2u, row 2u + 1) as one 4-byte store
      const int pr = pad16(2 * (j * (kP2Cols * 64) + static_cast<int>(threadIdx.x)));
      const uint32_t r0w[2] = {nx[j].x, nx[j].y}, r1w[2] = {nx[j].z, nx[j].w};
#pragma unroll
      for (int e = 0; e < kP2Cols; ++e) {
        const uint32_t lo = (e & 1) ? (r0w[e >> 1] >> 16) : (r0w[e >> 1] & 0xFFFFu);
        const uint32_t hi = (e & 1) ? (r1w[e >> 1] & 0xFFFF0000u) : (r1w[e >> 1] << 16);
        *reinterpret_cast<uint32_t*>(cols + e * kColArr + pr) = lo | hi;
      }
    }
    __syncthreads();
    // the term's factors are loaded before the next tile (loads retire in
    // order), so the products wait for them and not for the prefetch, which
    // overlaps them (the scheduling barriers keep that order)
    const Fac16 f2 = fac16(a, t, 2, lane), f0 = fac16(a, t, 0, lane);
    const float4 f1v = fac32(a, t, 1, lane);
    __builtin_amdgcn_sched_barrier(0);
    load(min(t + 1, a.nterms - 1));   // branch-free: a wait after a branch would drain all loads
    __builtin_amdgcn_sched_barrier(0);
    const Fac16 f1 = split_scaled(f1v, a.lam[t]);
    // column w: blocks b = x1 with X[p = x2][q = x0], rows 256 c + 16 b + 4 g + i
    uint32_t u[16][2];
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      const u2v x = *reinterpret_cast<const u2v*>(mc + 16 * b);
      u[b][0] = x[0];
      u[b][1] = x[1];
    }
    aform16(u, f2);                    // (p = x0, q = y2)
    aform16(u, f0);                    // (p = y2, q = y0)
    exchange16(u);                     // blocks y2, (p = x1, q = y0)
#pragma unroll
    for (int b = 0; b < 16; ++b) {     // B(lambda T1) into the action's sum: (p = y1, q = y0)
      const s4v x = op(u[b][0], u[b][1]);
      acc[b] = mfma(f1.lo, x, acc[b]);
      acc[b] = mfma(f1.hi, x, acc[b]);
    }
    if (t + 1 == a.term_start[act + 1]) {
#pragma unroll
      for (int b = 0; b < 16; ++b) {
#pragma unroll
        for (int i = 0; i < 4; ++i) best[b][i] = acc[b][i] > best[b][i] ? acc[b][i] : best[b][i];
        acc[b] = f4v{0.f, 0.f, 0.f, 0.f};
      }
      ++act;
    }
  }
  // Eq. 1: V' = R + gamma (1 - terminal) (max_a P_a (V - cs) + cs); state of
  // lane (g, c), register (b, i): row 256 c + 16 (4 g + i) + b, column
  // tile * 8 + w
  double res = 0.0;
  const int col = tile * kTile + half * kP2Cols + w;
#pragma unroll
  for (int b = 0; b < 16; ++b) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int s = (256 * c + 16 * (4 * g + i) + b) * kFib + col;
      const float gm = is_terminal(a.term_bits, s) ? 0.f : a.gamma;
      const float vnew = fmaf(gm, best[b][i] + cs, a.R[s]);
      const double d = static_cast<double>(vnew) - static_cast<double>(a.V[s]);
      a.Vout[s] = vnew;
      res = nanmax(res, fabs(d));
    }
  }
  block_max_to_slot(res, a.res_slot);
}

// ------------------------------------------------------------------ FP32
// The same chain in FP32 on the 16 x 16 x 4 FP32 product (lane (g, c) gives
// A[c][g] and B[g][c] of a K = 4 slice; four slices make a 16 x 16 x 16
// product).  A block X[p][q] in the result layout (register i = X[4g + i][c])
// serves as slice q = i of either operand if the factor's slice q holds
// F[c][4g + q]: the product then contracts p in the order 4g + q, which is
// only a permutation of the summation.  Those factor registers are the same
// four values F[c][4g .. 4g + 3] as in the BF16 unit.  The exchange moves
// whole FP32 registers (no halves).  The intermediate is FP32 in tiles of 4
// columns (8 rows x 16 bytes = one line per pass-1 block and tile).
//   pass 1: 8 rows per block (LDS rows of 4096 + 4 per 256 floats, 16-byte
//     stores); pass 2: one tile (4 columns) per block, two blocks per CU, the
//     tile loaded at the start of each term (no register prefetch: at 64 FP32
//     values per lane it would not fit next to the sums; the other block's
//     matrix products cover the load).

constexpr int kTile32 = 4;                       // columns per FP32 tile
constexpr int kColArr32 = kFib + 16 * 4;         // 4160 floats
constexpr int kSlab32 = kColArr32 + 8;           // 4168: 8 rows x 2 tiles of a read on distinct banks

__device__ __forceinline__ int padf(int v) { return v + ((v >> 8) << 2); }

__device__ __forceinline__ f4v mfma4(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// A form, u[b] <- X_b^T F^T (F as four slices f[q] = F[c][4g + q]).
__device__ __forceinline__ void aform32(float (&u)[16][4], const float4& f) {
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    f4v d = {0.f, 0.f, 0.f, 0.f};
    d = mfma4(u[b][0], f.x, d);
    d = mfma4(u[b][1], f.y, d);
    d = mfma4(u[b][2], f.z, d);
    d = mfma4(u[b][3], f.w, d);
#pragma unroll
    for (int i = 0; i < 4; ++i) u[b][i] = d[i];
  }
}

// 4 x 4 transpose of lane groups against the four registers.
__device__ __forceinline__ void lane_group_transpose(float (&x)[4]) {
  uint32_t y[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) y[m] = __float_as_uint(x[m]);
  auto s02 = __builtin_amdgcn_permlane32_swap(y[0], y[2], false, false);
  auto s13 = __builtin_amdgcn_permlane32_swap(y[1], y[3], false, false);
  auto s01 = __builtin_amdgcn_permlane16_swap(s02[0], s13[0], false, false);
  auto s23 = __builtin_amdgcn_permlane16_swap(s02[1], s13[1], false, false);
  x[0] = __uint_as_float(s01[0]);
  x[1] = __uint_as_float(s01[1]);
  x[2] = __uint_as_float(s23[0]);
  x[3] = __uint_as_float(s23[1]);
}

// u[b][i] = X[b][4g + i][c]  ->  X'[b][p][c] = X[p][b][c].  Group (I, L):
// registers u[4m + I][L] (m = 0..3) transposed against the lane groups land
// in u[4k + L][I]; groups (I, L) and (L, I) trade places, (I, I) stay.
__device__ __forceinline__ void exchange32(float (&u)[16][4]) {
#pragma unroll
  for (int I = 0; I < 4; ++I) {
#pragma unroll
    for (int L = I; L < 4; ++L) {
      float x[4], y[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        x[m] = u[4 * m + I][L];
        y[m] = u[4 * m + L][I];
      }
      lane_group_transpose(x);
      if (L != I) lane_group_transpose(y);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        u[4 * k + L][I] = x[k];
        if (L != I) u[4 * k + I][L] = y[k];
      }
    }
  }
}

__global__ __launch_bounds__(kP1Rows * 64) void chain16f_pass1(ChainArgs<float> a) {
  __shared__ __align__(16) float slab[kP1Rows * kSlab32];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int r0 = xcd_block(blockIdx.x, gridDim.x) * kP1Rows;
  const float cs = a.shift_keys ? midrange(a.shift_keys) : 0.f;
  float v[16][4];   // row r0 + w: blocks b = x3, X[p = x4][q = x5]
  {
    const float* Vr = a.V + static_cast<int64_t>(r0 + w) * kFib + 64 * g + c;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
#pragma unroll
      for (int i = 0; i < 4; ++i) v[b][i] = Vr[256 * b + 16 * i] - cs;
    }
  }
  float* my = slab + w * kSlab32 + padf(256 * c + 4 * g);
  const int64_t S = a.g.S, Rr = a.g.Rr;
  // the next term's factors are loaded just before this term's stores (see
  // the BF16 pass 1)
  float4 f3 = fac32(a, 0, 3, lane), f4 = fac32(a, 0, 4, lane), f5 = fac32(a, 0, 5, lane);
  for (int t = 0; t < a.nterms; ++t) {
    float u[16][4];
#pragma unroll
    for (int b = 0; b < 16; ++b) {     // A(T4): (p = x5, q = y4)
      f4v d = {0.f, 0.f, 0.f, 0.f};
      d = mfma4(v[b][0], f4.x, d);
      d = mfma4(v[b][1], f4.y, d);
      d = mfma4(v[b][2], f4.z, d);
      d = mfma4(v[b][3], f4.w, d);
#pragma unroll
      for (int i = 0; i < 4; ++i) u[b][i] = d[i];
    }
    aform32(u, f5);                    // (p = y4, q = y5)
    exchange32(u);                     // blocks y4, (p = x3, q = y5)
    aform32(u, f3);                    // (p = y5, q = y3): column 256 c + 16 b + 4 g + i
#pragma unroll
    for (int b = 0; b < 16; ++b)
      *reinterpret_cast<float4*>(my + 16 * b) = make_float4(u[b][0], u[b][1], u[b][2], u[b][3]);
    __syncthreads();
    {
      const int tn = min(t + 1, a.nterms - 1);
      f3 = fac32(a, tn, 3, lane);
      f4 = fac32(a, tn, 4, lane);
      f5 = fac32(a, tn, 5, lane);
    }
    __builtin_amdgcn_sched_barrier(0);
    float* Wt = a.W + static_cast<int64_t>(t) * S;
    constexpr int kUnits = (kFib / kTile32) * kP1Rows;   // 16-byte units of the block
#pragma unroll
    for (int j = 0; j < kUnits / (kP1Rows * 64); ++j) {
      const int q = threadIdx.x + j * (kP1Rows * 64);
      const int tl = q / kP1Rows, ww = q % kP1Rows;
      const float4 val = *reinterpret_cast<const float4*>(slab + ww * kSlab32 + padf(kTile32 * tl));
      *reinterpret_cast<float4*>(Wt + (static_cast<int64_t>(tl) * Rr + r0 + ww) * kTile32) = val;
    }
    __syncthreads();
  }
}

// two waves per SIMD: two blocks of four waves per CU
__global__ __launch_bounds__(kTile32 * 64, 2) void chain16f_pass2(ChainArgs<float> a) {
  __shared__ __align__(16) float cols[kTile32 * kColArr32];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int64_t S = a.g.S;
  // rows 2u and 2u + 1 of the tile (32 contiguous bytes), u = j * 256 + thread
  const float* Wb = a.W + static_cast<int64_t>(tile) * kFib * kTile32 + threadIdx.x * 2 * kTile32;
  constexpr int kUnits = kFib / 2 / (kTile32 * 64);
  f4v acc[16], best[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    acc[b] = f4v{0.f, 0.f, 0.f, 0.f};
    best[b] = f4v{-INFINITY, -INFINITY, -INFINITY, -INFINITY};
  }
  const float cs = a.shift_keys ? midrange(a.shift_keys) : 0.f;
  const float* mc = cols + w * kColArr32 + padf(256 * c + 4 * g);
  int act = 0;
  for (int t = 0; t < a.nterms; ++t) {
    // factors first (loads retire in order), then the tile
    const float4 f2 = fac32(a, t, 2, lane), f0 = fac32(a, t, 0, lane), f1v = fac32(a, t, 1, lane);
    __builtin_amdgcn_sched_barrier(0);
    float4 ld[kUnits][2];
    {
      const float* p = Wb + static_cast<int64_t>(t) * S;
#pragma unroll
      for (int j = 0; j < kUnits; ++j) {
        ld[j][0] = *reinterpret_cast<const float4*>(p + j * (kTile32 * 64) * 2 * kTile32);
        ld[j][1] = *reinterpret_cast<const float4*>(p + j * (kTile32 * 64) * 2 * kTile32 + kTile32);
      }
    }
    __syncthreads();   // the previous term's column reads are done
#pragma unroll
    for (int j = 0; j < kUnits; ++j) {
      const int pr = padf(2 * (j * (kTile32 * 64) + static_cast<int>(threadIdx.x)));
      *reinterpret_cast<float2*>(cols + 0 * kColArr32 + pr) = make_float2(ld[j][0].x, ld[j][1].x);
      *reinterpret_cast<float2*>(cols + 1 * kColArr32 + pr) = make_float2(ld[j][0].y, ld[j][1].y);
      *reinterpret_cast<float2*>(cols + 2 * kColArr32 + pr) = make_float2(ld[j][0].z, ld[j][1].z);
      *reinterpret_cast<float2*>(cols + 3 * kColArr32 + pr) = make_float2(ld[j][0].w, ld[j][1].w);
    }
    __syncthreads();
    const float lam = a.lam[t];
    const float4 f1 = make_float4(lam * f1v.x, lam * f1v.y, lam * f1v.z, lam * f1v.w);
    // column w: blocks b = x1 with X[p = x2][q = x0], rows 256 c + 16 b + 4 g + i
    float u[16][4];
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      const float4 x = *reinterpret_cast<const float4*>(mc + 16 * b);
      u[b][0] = x.x;
      u[b][1] = x.y;
      u[b][2] = x.z;
      u[b][3] = x.w;
    }
    aform32(u, f2);                    // (p = x0, q = y2)
    aform32(u, f0);                    // (p = y2, q = y0)
    exchange32(u);                     // blocks y2, (p = x1, q = y0)
#pragma unroll
    for (int b = 0; b < 16; ++b) {     // B(lambda T1) into the action's sum: (p = y1, q = y0)
      acc[b] = mfma4(f1.x, u[b][0], acc[b]);
      acc[b] = mfma4(f1.y, u[b][1], acc[b]);
      acc[b] = mfma4(f1.z, u[b][2], acc[b]);
      acc[b] = mfma4(f1.w, u[b][3], acc[b]);
    }
    if (t + 1 == a.term_start[act + 1]) {
#pragma unroll
      for (int b = 0; b < 16; ++b) {
#pragma unroll
        for (int i = 0; i < 4; ++i) best[b][i] = acc[b][i] > best[b][i] ? acc[b][i] : best[b][i];
        acc[b] = f4v{0.f, 0.f, 0.f, 0.f};
      }
      ++act;
    }
  }
  // Eq. 1, as in the BF16 pass 2
  double res = 0.0;
  const int col = tile * kTile32 + w;
#pragma unroll
  for (int b = 0; b < 16; ++b) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int s = (256 * c + 16 * (4 * g + i) + b) * kFib + col;
      const float gm = is_terminal(a.term_bits, s) ? 0.f : a.gamma;
      const float vnew = fmaf(gm, best[b][i] + cs, a.R[s]);
      const double d = static_cast<double>(vnew) - static_cast<double>(a.V[s]);
      a.Vout[s] = vnew;
      res = nanmax(res, fabs(d));
    }
  }
  block_max_to_slot(res, a.res_slot);
}

}  // namespace

// Both groups three modes of exactly 16 states (16^6 grid split 3 + 3), the
// factors packed as 16 x 16 blocks, every action with at least one term.
bool chain16_bf16_ok(const ChainGeom& g) {
  if (g.n != 6 || g.n1 != 3 || g.Rr != kFib || g.C != kFib) return false;
  for (int k = 0; k < 6; ++k)
    if (g.size[k] != 16 || g.fac_off[k] != 256 * k) return false;
  return g.term_stride == 6 * 256;
}

// The intermediate needs nterms * S FP32 values (the FP32 chain's buffer).
// tm: start at pass 1, stop after pass 2.
void launch_chain16_f32(const ChainArgs<float>& a, hipStream_t st, const LaunchTiming* tm) {
  const LaunchTiming t1{tm ? tm->start : nullptr, nullptr};
  const LaunchTiming t2{nullptr, tm ? tm->stop : nullptr};
  klaunch(chain16f_pass1, dim3(kFib / kP1Rows), dim3(kP1Rows * 64), 0, st, tm ? &t1 : nullptr, a);
  klaunch(chain16f_pass2, dim3(kFib / kTile32), dim3(kTile32 * 64), 0, st, tm ? &t2 : nullptr, a);
}

// The intermediate needs nterms * S BF16 values (the FP32 chain's buffer
// holds twice that).  tm: start at pass 1, stop after pass 2.
void launch_chain16_bf16(const ChainArgs<float>& a, hipStream_t st, const LaunchTiming* tm) {
  const LaunchTiming t1{tm ? tm->start : nullptr, nullptr};
  const LaunchTiming t2{nullptr, tm ? tm->stop : nullptr};
  klaunch(chain16_pass1, dim3(kFib / kP1Rows), dim3(kP1Rows * 64), 0, st, tm ? &t1 : nullptr, a);
  klaunch(chain16_pass2, dim3(kFib / kP2Cols), dim3(kP2Cols * 64), 0, st, tm ? &t2 : nullptr, a);   // two per tile
}

}  // namespace cpm

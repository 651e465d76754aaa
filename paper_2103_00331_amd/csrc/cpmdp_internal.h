// Internal declarations of the cpmdp GPU library (host runtime <-> kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "cpmdp.h"

namespace cpm {

constexpr int kMaxDims = 8;
constexpr int kMaxActions = 255;
constexpr int kSlots = 256;        // residual slots (one per sweep of a chunk)
constexpr int kSpread = 64;        // words per residual slot (atomics spread)
constexpr int kMaxBlocks = 2048;   // persistent grid: 256 CUs x 8 blocks
constexpr int kBlock = 256;        // threads per block of the streaming kernels
constexpr int kXcds = 8;           // MI355X: 8 XCDs, 32 CUs each
constexpr double kTieRel = 1e-12;  // tie tolerance relative to max(1,||V||)
constexpr int64_t kMarchMinPlane = 65536;  // plane size (states) from which the stencil marches
constexpr int kCertifiedRounds = 3;  // PI: certified improvement rounds before stopping

// Kind of one factor T^{(k)}_{a,r}.
enum FactorKind : uint8_t { F_IDENT = 0, F_SHIFT_P = 1, F_SHIFT_M = 2, F_DENSE = 3 };

// What a sweep writes.
//   MAX    : V'(s) = max_a Q_a(s); residual max |V' - V|.
//   GREEDY : as MAX, plus pi(s) by the tie rule; with an incumbent policy the
//            incumbent is kept unless beaten by more than tol, and the number
//            of changed states is counted.
//   EVAL   : V'(s) = R(s) + gamma (1 - tau(s)) (P_{pi(s)} V)(s).
//   RESID  : as EVAL but writes r(s) = V'(s) - V(s) as FP32 (refinement
//            right-hand side); residual max |r|.
enum Mode : int { MODE_MAX = 0, MODE_GREEDY = 1, MODE_EVAL = 2, MODE_RESID = 3 };

// Division by a runtime constant d < 2^31 for numerators < 2^31:
// q = (umulhi(n, magic) + n) >> shift   (Granlund & Montgomery, PLDI 1994).
struct FastDiv {
  uint32_t magic;
  uint32_t shift;
};

FastDiv make_fastdiv(uint32_t d);

// Row-major grid geometry.  size[] and stride[] describe the stored layout;
// `last` is the number of real states along the last dimension: a layout
// whose rows are padded to a multiple of 4 has size[n-1] > last, the padded
// entries are never read by a real state and never count in a residual.
struct GridGeom {
  int32_t n;
  int32_t S;
  int32_t size[kMaxDims];
  int32_t stride[kMaxDims];
  FastDiv div[kMaxDims];
  int32_t last;
  int32_t pad_;
};

// Optional events around one launch (hipExtLaunchKernelGGL records the
// kernel's own start / stop times in them): used to time single kernels.
struct LaunchTiming {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};

// ---------------------------------------------------------------- stencil
template <typename T>
struct StencilArgs {
  GridGeom g;
  int32_t A;
  int32_t npts;                 // 2n + 1: centre, then (+e_k, -e_k) per dim
  const T* w;                   // [A][npts] summed rank weights
  const T* wbase;               // [npts] weight shared by most actions per point
  const T* wdiff;               // [A][npts] w - wbase (mostly zero)
  int32_t states_per_block;     // contiguous states per block (multiple of 256*VEC)
  const T* V;                   // input values
  T* Vout;                      // MAX / GREEDY / EVAL output (nullable for GREEDY)
  const T* R;                   // rewards, or the right-hand side of a correction sweep
  const float* Rf;              // EVAL on a T=float sweep with FP32 rhs (== R) -- unused otherwise
  const uint32_t* term_bits;    // terminal mask, 1 bit per state
  const uint16_t* obs;          // per state, bit 2k / 2k+1: the +e_k / -e_k
                                // neighbour is an obstacle (nullptr: none)
  T gamma;
  const int32_t* pi_in;         // EVAL: policy; GREEDY: incumbent (nullable)
  int32_t* pi_out;              // GREEDY output (nullable)
  float* r_out;                 // RESID output
  const unsigned long long* vmax_bits;  // GREEDY: ||V||_inf as FP64 bits
  unsigned long long* res_slot; // max |out - V| as FP64 bits (atomic max)
  double* res_part;             // if set: block b stores its max at res_part[b]
                                // instead (res_slot unused)
  unsigned int* change_count;   // GREEDY with incumbent
  int32_t nblocks;
  int32_t vec;                  // states per thread along the last dim (1 or 4)
  int32_t march;                // 1: marching form (needs n >= 2 and vec == 4)
  int32_t march_tiles;          // plane tiles of 4 * kBlock states
  int32_t march_seg;            // planes per block
  int32_t axis;                 // 1: axis-structured weights (see stencil.hip)
  // Weights by value: kernel arguments are scalar-loaded, so the
  // wave-uniform weights sit in SGPRs.
  T kw_base[2 * kMaxDims + 1];
  T kw_axis[2 * kMaxDims * 3];  // per action: diff at centre, +axis, -axis
};

template <typename T>
void launch_stencil(const StencilArgs<T>& a, int mode, hipStream_t st,
                    const LaunchTiming* tm = nullptr);

// ------------------------------------------- Tensor-Train transition models
// One bonded mode product X^{(k+1)} (b_in channels of S) -> X^{(k)} (b_out
// channels) along dim k; core in the padded device layout Gd[r][j][l][i]
// (i, j padded to mm, l to lpad, zeros in the padding).
template <typename T>
struct TTStepArgs {
  const T* in;
  T* out;
  const T* core;
  int32_t S;
  int32_t m, mm;                // m_k and its padded size (4, 8 or 16)
  int32_t post;                 // prod_{j>k} m_j (stride of dim k)
  FastDiv post_div;
  int32_t positions;            // S / m_k fiber positions
  int32_t b_in, b_out, lpad;    // bonds b_{k+1}, b_k; b_k padded to a multiple of 4
};

// Eq. 1 over Y[a] = P_a V, fused with the max / argmax, policy value or
// policy residual (modes as for the other sweeps).
template <typename T>
struct TTEpiArgs {
  int32_t S, A;
  const T* Y;                   // [A][S]
  const T* V;
  T* Vout;
  const T* R;
  const uint32_t* term_bits;
  T gamma;
  const int32_t* pi_in;
  int32_t* pi_out;
  float* r_out;
  const unsigned long long* vmax_bits;
  unsigned long long* res_slot;
  unsigned int* change_count;
};

template <typename T>
void launch_tt_step(const TTStepArgs<T>& a, hipStream_t st, const LaunchTiming* tm = nullptr);

// The last two bonded mode products in one launch (FP32, m_{n-1} = m_{n-2}
// = 16): V (one channel) -> b_{n-2} channels, the b_{n-1} channels between
// them kept on chip.  Cores in the padded device layout of TTStepArgs.
struct TTStep2Args {
  const float* in;
  float* out;
  const float* core1;           // G_{n-1}: [1][16][lpad1][16]
  const float* core2;           // G_{n-2}: [b_mid][16][lpad2][16]
  int32_t S;
  int32_t b_mid, b_out, lpad1, lpad2;   // b_{n-1}, b_{n-2}, padded to multiples of 4
};
bool tt_last2_fits(const TTStep2Args& a);
void launch_tt_last2(const TTStep2Args& a, hipStream_t st, const LaunchTiming* tm = nullptr);
template <typename T>
void launch_tt_epilogue(const TTEpiArgs<T>& a, int mode, hipStream_t st,
                        const LaunchTiming* tm = nullptr);

// ---------------------------------------------------- Def. 3 successor lists
// Sliced layout with 64-state slices (one slice per wave): for slice q and
// action a the columns col_ptr[q*A + a] .. col_ptr[q*A + a + 1] hold the
// slice's lists for a, entry of lane l in column c at c * 64 + l (padding:
// probability 0).
constexpr int kSlice = 64;

template <typename T>
struct ListsArgs {
  int32_t S, A, nslices;
  int32_t slices_per_block;     // contiguous slices per block
  const int32_t* col_ptr;       // [nslices * A + 1]
  const int32_t* succ;          // [columns * 64]
  const T* prob;                // [columns * 64]
  const T* V;
  T* Vout;
  const T* R;
  const uint32_t* term_bits;
  T gamma;
  const int32_t* pi_in;
  int32_t* pi_out;
  float* r_out;
  const unsigned long long* vmax_bits;
  unsigned long long* res_slot;
  double* res_part;             // if set: per-block residual words (no atomics)
  unsigned int* change_count;
  int32_t nblocks;
};

template <typename T>
void launch_lists(const ListsArgs<T>& a, int mode, hipStream_t st,
                  const LaunchTiming* tm = nullptr);

// ----------------------------------------------------------- dense chains
struct ChainGeom {
  int32_t n, n1;                // dims [0, n1) = row group, [n1, n) = column group
  int32_t S, Rr, C;             // rows (prod of row dims), columns (prod of col dims)
  int32_t CT, ct_shift;         // columns per pass-2 tile (power of two)
  int32_t ntiles;               // ceil(C / CT)
  int32_t size[kMaxDims];
  int32_t fac_off[kMaxDims];    // offset of dim k's block inside one term
  int32_t term_stride;          // sum_k m_k^2
  int32_t mmax_row, mmax_col;
  int64_t w_term_stride;        // elements per term in the intermediate buffer
  FastDiv idiv[kMaxDims];       // division by mode k's stride in its LDS array
                                // (pass 2 for k < n1, pass 1 for k >= n1)
  int32_t r1;                   // pass 1 rows per block (one per wave), 0: one
                                // row per block with the slab in LDS
};

template <typename T>
struct ChainArgs {
  ChainGeom g;
  int32_t A;
  int32_t nterms;
  const int32_t* term_start;    // [A+1] first term of each action
  const T* fac;                 // packed factors in T
  const uint16_t* facbf;        // the same factors split into BF16 hi + lo
  const uint16_t* facbf_lo;     // (bit patterns; hi + lo = the FP32 factor)
  const T* lam;                 // [nterms]
  const uint8_t* kinds;         // [nterms][n]
  const T* V;
  T* W;                         // intermediates [nterms][ntiles][Rr][CT]
  T* Vout;
  const T* R;
  const uint32_t* term_bits;
  T gamma;
  const int32_t* pi_in;
  int32_t* pi_out;
  float* r_out;
  const unsigned long long* vmax_bits;
  unsigned long long* res_slot;
  unsigned int* change_count;
  // Keys [max V, max -V] of the input, or null.  When set, the chain runs on
  // V - c with c the midrange of V and adds c back (exact for stochastic
  // operators, and it keeps low-precision operands small).
  const unsigned long long* shift_keys;
};

// Unit of a chain's mode products: vector ALUs, FP32 or FP64 matrix cores,
// or BF16 operands on matrix cores with FP32 accumulation (matrix cores for
// modes with m_k <= 16 only; larger modes run on the vector ALUs in the
// chain's precision).  The BF16 unit splits every operand into hi + lo BF16
// parts and sums the products hi*hi + hi*lo + lo*hi.
enum ChainUnit { CHAIN_VALU = 0, CHAIN_F32_MFMA = 1, CHAIN_BF16 = 2, CHAIN_F64_MFMA = 3 };

template <typename T>
void launch_chain(const ChainArgs<T>& a, int mode, int unit, hipStream_t st,
                  const LaunchTiming* tm = nullptr);

// Register-resident BF16 and FP32 chains (max sweeps of 16^6 grids, split
// 3 + 3): their geometry test and launchers (chain16.hip).
bool chain16_bf16_ok(const ChainGeom& g);
void launch_chain16_bf16(const ChainArgs<float>& a, hipStream_t st, const LaunchTiming* tm);
void launch_chain16_f32(const ChainArgs<float>& a, hipStream_t st, const LaunchTiming* tm);

// ---------------------------------------------------------------- helpers
void launch_fill_u64(unsigned long long* p, int n, unsigned long long v, hipStream_t st);
void launch_fill_u32(unsigned int* p, int n, unsigned int v, hipStream_t st);
void launch_f64_to_f32(const double* src, float* dst, int64_t n, hipStream_t st);
void launch_f32_to_f64(const float* src, double* dst, int64_t n, hipStream_t st);
void launch_add_f32_to_f64(double* dst, const float* e, int64_t n, hipStream_t st);
void launch_fill_f32(float* p, int64_t n, float v, hipStream_t st);
void launch_copy_i32(const int32_t* src, int32_t* dst, int64_t n, hipStream_t st);
// slots[j * kSpread] = max of parts[j * nb .. j * nb + nb) as FP64 bits,
// for j < k (the other words of each slot are left alone).
void launch_reduce_parts(const double* parts, int nb, int k, unsigned long long* slots,
                         hipStream_t st);
void launch_maxabs_f64(const double* v, int64_t n, unsigned long long* slot, hipStream_t st);
void launch_shift_bounds(const double* V, const double* BV, const uint32_t* tbits, int64_t n,
                         unsigned long long* keys, hipStream_t st);
void launch_minmax_keys_f32(const float* V, int64_t n, unsigned long long* keys, hipStream_t st);
void launch_apply_shift(double* V, const double* BV, const uint32_t* tbits, int64_t n, double shift,
                        hipStream_t st);
void launch_check_policy(const int32_t* pi, int64_t n, int32_t A, unsigned int* bad, hipStream_t st);

}  // namespace cpm

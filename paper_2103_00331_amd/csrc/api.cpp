// Host runtime behind include/cpmdp.h: validation, factor classification,
// packing, workspace layout, and the value- / policy-iteration drivers.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "cpmdp_internal.h"
#include "handle.h"

namespace cpm {

FastDiv make_fastdiv(uint32_t d) {
  FastDiv f{};
  uint32_t l = 0;
  while ((1ull << l) < d) ++l;
  const uint64_t m = ((1ull << 32) * ((1ull << l) - d)) / d + 1;
  f.magic = static_cast<uint32_t>(m);
  f.shift = l;
  return f;
}

thread_local std::string g_last_error;

int fail(cpmdp_t* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  g_last_error = msg;
  return code;
}

#define HIP_TRY(h, call)                                                           \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail((h), CPMDP_E_DEVICE,                                             \
                  std::string(#call) + ": " + hipGetErrorString(e_));              \
  } while (0)

// ------------------------------------------------------------ validation

static int classify(const double* T, int m) {
  bool ident = true, sp = true, sm = true;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const double v = T[i * m + j];
      const double e_id = (i == j) ? 1.0 : 0.0;
      const double e_sp = (j == std::min(i + 1, m - 1)) ? 1.0 : 0.0;
      const double e_sm = (j == std::max(i - 1, 0)) ? 1.0 : 0.0;
      ident = ident && v == e_id;
      sp = sp && v == e_sp;
      sm = sm && v == e_sm;
    }
  if (ident) return F_IDENT;
  if (sp) return F_SHIFT_P;
  if (sm) return F_SHIFT_M;
  return F_DENSE;
}

// LDS per workgroup on gfx950 (160 KiB); a little is kept for the kernels'
// static arrays.
constexpr int64_t kLdsBytes = 160 * 1024;

// LDS bytes the chain kernels of geometry g request per workgroup.
int64_t chain_lds_bytes(const ChainGeom& g, size_t b) {
  const int64_t TE = static_cast<int64_t>(g.Rr) * g.CT;
  // pass 2: the tile, plus (FP32 chains on the matrix cores) the row-group
  // factors of one term staged as FP32 or as BF16 hi + lo
  const int64_t rows_len = (g.n1 < g.n) ? g.fac_off[g.n1] : g.term_stride;
  const int64_t p2 = static_cast<int64_t>(b) * (TE + (TE >> 4) + 2 + rows_len) + 1024 + 256;
  const int64_t cols_len = g.term_stride - ((g.n1 < g.n) ? g.fac_off[g.n1] : g.term_stride);
  const int64_t p1 = (g.n1 == g.n) ? 0
                     : (g.r1 > 0) ? static_cast<int64_t>(b) * (g.r1 * (g.C + (g.C >> 4) + 1) +
                                                               cols_len) + 512
                                  : static_cast<int64_t>(b) * (2 * (g.C + (g.C >> 4) + 1) + 2) + 256;
  return std::max(p1, p2);
}

// Split the dims into a row group [0, n1) and a column group [n1, n) so that
// a pass-1 row slab (two copies) and a pass-2 tile (rows x CT) fit in LDS;
// prefer balanced groups.  te_max also bounds the per-thread register state
// of pass 2 (16384 / 1024 threads = 16 elements; FP64: 8).
static bool choose_split(const std::vector<int64_t>& sizes, int64_t S, size_t b,
                         ChainGeom& g) {
  const int n = static_cast<int>(sizes.size());
  const int64_t te_max = std::min<int64_t>(b == 8 ? 8192 : 16384,
                                           (kLdsBytes - 4096) / static_cast<int64_t>(b));
  const int64_t c_max =
      static_cast<int64_t>((kLdsBytes - 4096) / (2.0 * b * (1.0 + 1.0 / 16.0))) - 4;
  int64_t mmax = 0;
  for (auto m : sizes) mmax = std::max(mmax, m);
  if (mmax > 32) return false;
  int best_n1 = -1;
  double best_score = 1e30;
  if (S <= 4096) {
    best_n1 = n;
  } else {
    int64_t Rr = 1;
    for (int n1 = 1; n1 < n; ++n1) {
      Rr *= sizes[n1 - 1];
      const int64_t C = S / Rr;
      if (C > c_max || Rr > te_max) continue;
      const double score = std::fabs(std::log2(static_cast<double>(Rr)) -
                                     std::log2(static_cast<double>(C)));
      if (score < best_score - 1e-9) {
        best_score = score;
        best_n1 = n1;
      }
    }
    if (best_n1 < 0 && S <= te_max) best_n1 = n;
  }
  if (best_n1 < 0) return false;
  std::memset(&g, 0, sizeof(g));
  g.n = n;
  g.n1 = best_n1;
  g.S = static_cast<int32_t>(S);
  int64_t Rr = 1;
  for (int k = 0; k < best_n1; ++k) Rr *= sizes[k];
  g.Rr = static_cast<int32_t>(Rr);
  g.C = static_cast<int32_t>(S / Rr);
  int ct = 1, sh = 0;
  while (ct < 64 && Rr * ct * 2 <= te_max && ct < g.C) {
    ct *= 2;
    ++sh;
  }
  g.CT = ct;
  g.ct_shift = sh;
  g.ntiles = (g.C + ct - 1) / ct;
  int off = 0;
  for (int k = 0; k < n; ++k) {
    g.size[k] = static_cast<int32_t>(sizes[k]);
    g.fac_off[k] = off;
    off += static_cast<int32_t>(sizes[k] * sizes[k]);
  }
  g.term_stride = off;
  g.mmax_row = 0;
  g.mmax_col = 0;
  for (int k = 0; k < n; ++k) {
    if (k < best_n1) g.mmax_row = std::max<int32_t>(g.mmax_row, g.size[k]);
    else g.mmax_col = std::max<int32_t>(g.mmax_col, g.size[k]);
  }
  g.w_term_stride = (best_n1 == n) ? 0 : static_cast<int64_t>(g.ntiles) * g.Rr * g.CT;
  int64_t inner = g.CT;               // pass 2: X is [row dims][CT]
  for (int k = best_n1 - 1; k >= 0; --k) {
    g.idiv[k] = make_fastdiv(static_cast<uint32_t>(inner));
    inner *= sizes[k];
  }
  inner = 1;                          // pass 1: the slab is [column dims]
  for (int k = n - 1; k >= best_n1; --k) {
    g.idiv[k] = make_fastdiv(static_cast<uint32_t>(inner));
    inner *= sizes[k];
  }
  // pass 1 with one row per wave: as many rows (<= 8, a power of two) as
  // fit in LDS, the row kept in registers (at most 64 values per lane)
  g.r1 = 0;
  if (best_n1 < n && g.C <= 64 * 64) {
    const int64_t cols_len = g.term_stride - g.fac_off[best_n1];
    for (int r1 = 8; r1 >= 2; r1 /= 2) {
      const int64_t lds = static_cast<int64_t>(b) * (r1 * (g.C + (g.C >> 4) + 1) + cols_len) + 512;
      if (lds <= kLdsBytes && r1 <= g.Rr) {
        g.r1 = r1;
        break;
      }
    }
  }
  return true;
}

// ------------------------------------------------------------- workspace

static size_t align_up(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

struct Carver {
  char* base;
  size_t off = 0;
  template <typename P>
  P* take(size_t count) {
    P* p = base ? reinterpret_cast<P*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(P));
    return p;
  }
};

void layout(const cpmdp_t* h, DevPtrs* dp, char* base, size_t* total) {
  Carver cv{base};
  const size_t S = static_cast<size_t>(h->S);
  const size_t A = static_cast<size_t>(h->A);
  const size_t T = h->lambdas.size();
  DevPtrs& d = *dp;
  d.R64 = cv.take<double>(S);
  d.R32 = cv.take<float>(S);
  d.tbits = cv.take<uint32_t>((S + 31) / 32 + 1);
  d.slots = cv.take<unsigned long long>(static_cast<size_t>(kSlots) * kSpread);
  d.vmax = cv.take<unsigned long long>(8);   // [0] max|V|, [2..3] bound shift, [4..5] chain shift
  d.counters = cv.take<unsigned int>(8);
  d.Va64 = cv.take<double>(S);
  d.Va32 = cv.take<float>(S);
  d.Vb32 = cv.take<float>(S);
  d.E0 = cv.take<float>(S);
  d.E1 = cv.take<float>(S);
  d.r32 = cv.take<float>(S);
  d.piA = cv.take<int32_t>(S);
  if (h->path == CPMDP_PATH_LISTS) {
    const size_t ent = h->l_succ.size();
    d.l_cols = cv.take<int32_t>(h->l_cols.size());
    d.l_succ = cv.take<int32_t>(ent);
    d.l_p64 = cv.take<double>(ent);
    d.l_p32 = cv.take<float>(ent);
    d.parts = cv.take<double>(static_cast<size_t>(kSlots) * h->l_blocks);
    d.W = nullptr;
  } else if (h->path == CPMDP_PATH_TT) {
    d.t_core64 = cv.take<double>(h->t_core.size());
    d.t_core32 = cv.take<float>(h->t_core.size());
    d.t_X0 = cv.take<char>(static_cast<size_t>(h->t_maxb) * S * sizeof(double));
    d.t_X1 = cv.take<char>(static_cast<size_t>(h->t_maxb) * S * sizeof(double));
    d.t_Y = cv.take<char>(A * S * sizeof(double));
    d.W = nullptr;
  } else if (h->path == CPMDP_PATH_STENCIL) {
    const size_t P = 2 * static_cast<size_t>(h->n) + 1;
    d.w64 = cv.take<double>(3 * A * P);   // w, wdiff [A][P], then wbase [P]
    d.w32 = cv.take<float>(3 * A * P);
    d.parts = cv.take<double>(static_cast<size_t>(kSlots) *
                              std::max(h->st_blocks, h->st_march_blocks));
    d.obs = h->obstacle.empty() ? nullptr : cv.take<uint16_t>(S);
    d.fac64 = nullptr;
    d.fac32 = nullptr;
    d.facbf = nullptr;
    d.W = nullptr;
  } else {
    const size_t F = T * static_cast<size_t>(h->cg64.term_stride);
    d.fac64 = cv.take<double>(F);
    d.fac32 = cv.take<float>(F);
    d.facbf = cv.take<uint16_t>(2 * F);   // BF16 split: hi [F], then lo [F]
    d.lam64 = cv.take<double>(T);
    d.lam32 = cv.take<float>(T);
    d.kinds = cv.take<uint8_t>(T * h->n);
    d.term_start = cv.take<int32_t>(A + 1);
    const size_t w64 = T * static_cast<size_t>(h->cg64.w_term_stride) * sizeof(double);
    const size_t w32 = T * static_cast<size_t>(h->cg32.w_term_stride) * sizeof(float);
    d.W = cv.take<char>(std::max<size_t>(std::max(w64, w32), 256));
  }
  *total = cv.off;
}

// ---------------------------------------------------------------- sweeps

GridGeom make_geom(const cpmdp_t* h) {
  GridGeom g{};
  g.n = h->n;
  g.S = static_cast<int32_t>(h->S);
  int64_t st = 1;
  for (int k = h->n - 1; k >= 0; --k) {
    g.size[k] = static_cast<int32_t>(h->sizes[k]);
    g.stride[k] = static_cast<int32_t>(st);
    g.div[k] = make_fastdiv(static_cast<uint32_t>(h->sizes[k]));
    st *= h->sizes[k];
  }
  g.last = g.size[h->n - 1];
  return g;
}

// Kernel arguments of one stencil sweep in precision T (FP64 or FP32 copies
// of R and of the weights).
template <typename T>
static StencilArgs<T> stencil_args(cpmdp_t* h, const void* V, void* Vout, const void* R,
                                   const int32_t* pi_in, int32_t* pi_out, float* r_out,
                                   unsigned long long* slot, unsigned int* ctr,
                                   double* part) {
  constexpr bool f64 = std::is_same<T, double>::value;
  const size_t AP = static_cast<size_t>(h->A) * (2 * h->n + 1);
  const T* w = f64 ? reinterpret_cast<const T*>(h->d.w64) : reinterpret_cast<const T*>(h->d.w32);
  StencilArgs<T> a{};
  a.g = h->geom;
  a.A = h->A;
  a.npts = 2 * h->n + 1;
  a.w = w;
  a.wdiff = w + AP;
  a.wbase = w + 2 * AP;
  a.states_per_block = h->st_states_per_block;
  a.vec = h->st_vec;
  a.axis = h->st_axis;
  if (a.axis) {
    for (int i = 0; i < 2 * h->n + 1; ++i) a.kw_base[i] = static_cast<T>(f64 ? h->kw64[i] : h->kw32[i]);
    const size_t na = (f64 ? h->kw64.size() : h->kw32.size()) - (2 * h->n + 1);
    for (size_t i = 0; i < na; ++i)
      a.kw_axis[i] = static_cast<T>(f64 ? h->kw64[2 * h->n + 1 + i] : h->kw32[2 * h->n + 1 + i]);
  }
  a.V = static_cast<const T*>(V);
  a.Vout = static_cast<T*>(Vout);
  a.R = static_cast<const T*>(R);
  a.term_bits = h->d.tbits;
  a.obs = h->d.obs;
  a.gamma = static_cast<T>(h->gamma);
  a.pi_in = pi_in;
  a.pi_out = pi_out;
  a.r_out = r_out;
  a.vmax_bits = h->d.vmax;
  a.res_slot = slot;
  a.res_part = part;
  a.change_count = ctr;
  a.nblocks = h->st_blocks;
  if (h->st_march && h->opt_march) {
    a.march = 1;
    a.march_tiles = h->st_march_tiles;
    a.march_seg = h->st_march_seg;
    a.nblocks = h->st_march_blocks;
  }
  return a;
}

// One Tensor-Train sweep: per action the chain of bonded mode products
// (last dim first, the bond channels ping-ponging between X0 and X1, the
// last step writing Y[a] = P_a V), then the Eq. 1 epilogue over all Y[a].
// Timing events, when given, span the first step to the epilogue.
template <typename T>
static void tt_sweep(cpmdp_t* h, int mode, const void* V, void* Vout, const void* R,
                     const int32_t* pi_in, int32_t* pi_out, float* r_out,
                     unsigned long long* slot, unsigned int* ctr, const LaunchTiming* tm) {
  constexpr bool f64 = std::is_same<T, double>::value;
  const T* cores = f64 ? reinterpret_cast<const T*>(h->d.t_core64)
                       : reinterpret_cast<const T*>(h->d.t_core32);
  T* X[2] = {reinterpret_cast<T*>(h->d.t_X0), reinterpret_cast<T*>(h->d.t_X1)};
  T* Y = reinterpret_cast<T*>(h->d.t_Y);
  const int n = h->n;
  const int32_t S = static_cast<int32_t>(h->S);
  const LaunchTiming t_first{tm ? tm->start : nullptr, nullptr};
  const LaunchTiming t_last{nullptr, tm ? tm->stop : nullptr};
  bool first = true;
  for (int a = 0; a < h->A; ++a) {
    const T* cur = static_cast<const T*>(V);
    int which = 0;
    int k = n - 1;
    if constexpr (!f64) {
      // FP32 with two trailing modes of 16: both products in one launch
      if (n >= 2 && h->sizes[n - 1] == 16 && h->sizes[n - 2] == 16) {
        TTStep2Args s2{};
        s2.in = cur;
        s2.out = n == 2 ? Y + static_cast<size_t>(a) * S : X[which];
        s2.core1 = cores + h->t_off[static_cast<size_t>(a) * n + n - 1];
        s2.core2 = cores + h->t_off[static_cast<size_t>(a) * n + n - 2];
        s2.S = S;
        s2.b_mid = h->t_bonds[static_cast<size_t>(a) * (n + 1) + n - 1];
        s2.b_out = h->t_bonds[static_cast<size_t>(a) * (n + 1) + n - 2];
        s2.lpad1 = (s2.b_mid + 3) & ~3;
        s2.lpad2 = (s2.b_out + 3) & ~3;
        if (tt_last2_fits(s2)) {
          launch_tt_last2(s2, h->stream, (tm && first) ? &t_first : nullptr);
          first = false;
          cur = s2.out;
          which ^= 1;
          k = n - 3;
        }
      }
    }
    for (; k >= 0; --k) {
      TTStepArgs<T> s{};
      s.in = cur;
      s.out = k == 0 ? Y + static_cast<size_t>(a) * S : X[which];
      s.core = cores + h->t_off[static_cast<size_t>(a) * n + k];
      s.S = S;
      s.m = static_cast<int32_t>(h->sizes[k]);
      s.mm = h->t_mm[k];
      s.post = h->geom.stride[k];
      s.post_div = make_fastdiv(static_cast<uint32_t>(s.post));
      s.positions = S / s.m;
      s.b_in = h->t_bonds[static_cast<size_t>(a) * (n + 1) + k + 1];
      s.b_out = h->t_bonds[static_cast<size_t>(a) * (n + 1) + k];
      s.lpad = (s.b_out + 3) & ~3;
      launch_tt_step<T>(s, h->stream, (tm && first) ? &t_first : nullptr);
      first = false;
      cur = s.out;
      which ^= 1;
    }
  }
  TTEpiArgs<T> e{};
  e.S = S;
  e.A = h->A;
  e.Y = Y;
  e.V = static_cast<const T*>(V);
  e.Vout = static_cast<T*>(Vout);
  e.R = static_cast<const T*>(R);
  e.term_bits = h->d.tbits;
  e.gamma = static_cast<T>(h->gamma);
  e.pi_in = pi_in;
  e.pi_out = pi_out;
  e.r_out = r_out;
  e.vmax_bits = h->d.vmax;
  e.res_slot = slot;
  e.change_count = ctr;
  launch_tt_epilogue<T>(e, mode, h->stream, tm ? &t_last : nullptr);
}

int stencil_grid(const cpmdp_t* h) {
  if (h->path == CPMDP_PATH_LISTS) return h->l_blocks;
  return (h->st_march && h->opt_march) ? h->st_march_blocks : h->st_blocks;
}

// One sweep on the bound stream.  prec64 selects FP64 buffers (T = double)
// or FP32 (T = float).  V, Vout, R are typed by that choice.
void sweep(cpmdp_t* h, bool prec64, int mode, const void* V, void* Vout, const void* R,
           const int32_t* pi_in, int32_t* pi_out, float* r_out,
           unsigned long long* slot, unsigned int* ctr, bool bf16, const LaunchTiming* tm,
           double* part) {
  const hipStream_t st = h->stream;
  if (h->path == CPMDP_PATH_TT) {
    if (prec64) tt_sweep<double>(h, mode, V, Vout, R, pi_in, pi_out, r_out, slot, ctr, tm);
    else tt_sweep<float>(h, mode, V, Vout, R, pi_in, pi_out, r_out, slot, ctr, tm);
    return;
  }
  if (h->path == CPMDP_PATH_LISTS) {
    auto fill = [&](auto& a, auto* prob) {
      using T = std::remove_pointer_t<decltype(prob)>;
      a.S = static_cast<int32_t>(h->S);
      a.A = h->A;
      a.nslices = h->l_nslices;
      a.slices_per_block = h->l_slices_per_block;
      a.col_ptr = h->d.l_cols;
      a.succ = h->d.l_succ;
      a.prob = prob;
      a.V = static_cast<const T*>(V);
      a.Vout = static_cast<T*>(Vout);
      a.R = static_cast<const T*>(R);
      a.term_bits = h->d.tbits;
      a.gamma = static_cast<T>(h->gamma);
      a.pi_in = pi_in;
      a.pi_out = pi_out;
      a.r_out = r_out;
      a.vmax_bits = h->d.vmax;
      a.res_slot = slot;
      a.res_part = part;
      a.change_count = ctr;
      a.nblocks = h->l_blocks;
    };
    if (prec64) {
      ListsArgs<double> a{};
      fill(a, h->d.l_p64);
      launch_lists<double>(a, mode, st, tm);
    } else {
      ListsArgs<float> a{};
      fill(a, h->d.l_p32);
      launch_lists<float>(a, mode, st, tm);
    }
    return;
  }
  if (h->path == CPMDP_PATH_STENCIL) {
    if (prec64) {
      StencilArgs<double> a =
          stencil_args<double>(h, V, Vout, R, pi_in, pi_out, r_out, slot, ctr, part);
      launch_stencil<double>(a, mode, st, tm);
    } else {
      StencilArgs<float> a =
          stencil_args<float>(h, V, Vout, R, pi_in, pi_out, r_out, slot, ctr, part);
      launch_stencil<float>(a, mode, st, tm);
    }
    return;
  }
  if (prec64) {
    ChainArgs<double> a{};
    a.g = h->cg64;
    a.A = h->A;
    a.nterms = static_cast<int32_t>(h->lambdas.size());
    a.term_start = h->d.term_start;
    a.fac = h->d.fac64;
    a.lam = h->d.lam64;
    a.kinds = h->d.kinds;
    a.V = static_cast<const double*>(V);
    a.W = (a.g.n1 == a.g.n) ? const_cast<double*>(a.V) : reinterpret_cast<double*>(h->d.W);
    a.Vout = static_cast<double*>(Vout);
    a.R = static_cast<const double*>(R);
    a.term_bits = h->d.tbits;
    a.gamma = h->gamma;
    a.pi_in = pi_in;
    a.pi_out = pi_out;
    a.r_out = r_out;
    a.vmax_bits = h->d.vmax;
    a.res_slot = slot;
    a.change_count = ctr;
    a.facbf = nullptr;
    a.facbf_lo = nullptr;
    launch_chain<double>(a, mode, CHAIN_F64_MFMA, st, tm);
  } else {
    ChainArgs<float> a{};
    a.g = h->cg32;
    a.A = h->A;
    a.nterms = static_cast<int32_t>(h->lambdas.size());
    a.term_start = h->d.term_start;
    a.fac = h->d.fac32;
    a.lam = h->d.lam32;
    a.kinds = h->d.kinds;
    a.V = static_cast<const float*>(V);
    a.W = (a.g.n1 == a.g.n) ? const_cast<float*>(a.V) : reinterpret_cast<float*>(h->d.W);
    a.Vout = static_cast<float*>(Vout);
    a.R = static_cast<const float*>(R);
    a.term_bits = h->d.tbits;
    a.gamma = static_cast<float>(h->gamma);
    a.pi_in = pi_in;
    a.pi_out = pi_out;
    a.r_out = r_out;
    a.vmax_bits = h->d.vmax;
    a.res_slot = slot;
    a.change_count = ctr;
    a.facbf = h->d.facbf;
    a.facbf_lo = h->d.facbf + h->factors.size();
    if (bf16) {
      // BF16 operands: run the chain on V - midrange(V) (Sec. 2.2 operators
      // are row-stochastic, so P (V - c) + c = P V) to keep rounding small.
      launch_fill_u64(h->d.vmax + 4, 2, 0ull, st);
      launch_minmax_keys_f32(a.V, h->S, h->d.vmax + 4, st);
      a.shift_keys = h->d.vmax + 4;
    }
    launch_chain<float>(a, mode, bf16 ? CHAIN_BF16 : CHAIN_F32_MFMA, st, tm);
  }
}

static double bits_to_double(unsigned long long b) {
  double v;
  std::memcpy(&v, &b, sizeof(v));
  return v;
}

// Residual slot j of a chunk = kSpread words starting at slots + j * kSpread.
static unsigned long long* slot_of(cpmdp_t* h, int j) { return h->d.slots + static_cast<size_t>(j) * kSpread; }

static void zero_slots(cpmdp_t* h, int n) {
  launch_fill_u64(h->d.slots, n * kSpread, 0ull, h->stream);
}

// Read n residual slots (max over each slot's words) and optionally the
// counters back to the host.
static int read_slots(cpmdp_t* h, int n, std::vector<double>& out, unsigned* ctr0) {
  HIP_TRY(h, hipMemcpyAsync(h->host_slots, h->d.slots,
                            sizeof(unsigned long long) * static_cast<size_t>(n) * kSpread,
                            hipMemcpyDeviceToHost, h->stream));
  if (ctr0)
    HIP_TRY(h, hipMemcpyAsync(h->host_ctr, h->d.counters, sizeof(unsigned) * 2,
                              hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  out.resize(n);
  for (int i = 0; i < n; ++i) {
    unsigned long long m = 0;
    for (int j = 0; j < kSpread; ++j) m = std::max(m, h->host_slots[static_cast<size_t>(i) * kSpread + j]);
    out[i] = bits_to_double(m);
  }
  if (ctr0) *ctr0 = h->host_ctr[0];
  return CPMDP_OK;
}

static int check_device(cpmdp_t* h) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(h, CPMDP_E_DEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return CPMDP_OK;
}

// Chunk size for the next run of sweeps: enough to reach eps at the
// observed contraction rate, bounded to keep overshoot and host reads small.
// Sweeps still needed to bring res_last down to eps at the contraction rate
// observed over the last chunk (gamma until one is observed).
static double predict_need(double res_first, double res_last, int k_prev, double gamma,
                           double eps) {
  double rate = gamma;
  if (k_prev > 1 && res_first > 0 && res_last > 0 && std::isfinite(res_first) &&
      std::isfinite(res_last)) {
    rate = std::pow(res_last / res_first, 1.0 / (k_prev - 1));
    rate = std::min(std::max(rate, 0.3), 0.999999);
  }
  if (res_last > eps && std::isfinite(res_last))
    return std::ceil(std::log(eps / res_last) / std::log(rate));
  return 8.0;
}

// Chunked sweeps of one mode until the residual of a sweep <= tol.
// cur/alt: ping-pong buffers (cur holds the input on entry and the result on
// exit).  Returns status; *done = the last sweep's residual <= tol.
//
// Two chunks are kept in flight: while the host waits for one chunk's
// residuals (copied to pinned memory behind an event), the next chunk is
// already queued, so the device does not idle during the host's turnaround.
// The residual slots and per-block words are split in two halves, one per
// chunk in flight.  A chunk queued behind one that reached tol only runs
// more sweeps of the contraction; the reported residual is that of the last
// sweep run.
// Residual trend of a run of sweeps (first and last residual of its last
// chunk of k sweeps), handed from one stage of a solve to the next so that
// the next stage's first chunk is sized from it instead of probed.
struct SweepTrend {
  double rf = INFINITY, rl = INFINITY;
  int k = 0;
};

template <typename P>
static int run_sweeps(cpmdp_t* h, bool prec64, int mode, P*& cur, P*& alt, const void* R,
                      const int32_t* pi, double tol, double stall_floor, int64_t budget,
                      int64_t* sweeps, bool* done, double* last_res, bool bf16,
                      SweepTrend* trend = nullptr) {
  constexpr int kHalf = kSlots / 2;   // chunks hold at most 128 sweeps
  *done = false;
  // stencil and list sweeps leave one residual word per block, reduced per
  // chunk
  const bool parts = h->path == CPMDP_PATH_STENCIL || h->path == CPMDP_PATH_LISTS;
  const int nb = parts ? stencil_grid(h) : 0;
  struct Chunk {
    int half, k;
  };
  Chunk q[2];
  int nq = 0, next_half = 0;
  int64_t issued = *sweeps;
  auto issue = [&](int k) -> int {
    const int half = next_half;
    next_half ^= 1;
    unsigned long long* sl = h->d.slots + static_cast<size_t>(half) * kHalf * kSpread;
    double* pt = parts ? h->d.parts + static_cast<size_t>(half) * kHalf * nb : nullptr;
    launch_fill_u64(sl, k * kSpread, 0ull, h->stream);
    for (int j = 0; j < k; ++j) {
      sweep(h, prec64, mode, cur, alt, R, pi, nullptr, nullptr, sl + static_cast<size_t>(j) * kSpread,
            nullptr, bf16, nullptr, pt ? pt + static_cast<size_t>(j) * nb : nullptr);
      std::swap(cur, alt);
    }
    if (parts) launch_reduce_parts(pt, nb, k, sl, h->stream);
    int rc = check_device(h);
    if (rc) return rc;
    HIP_TRY(h, hipMemcpyAsync(h->host_slots + static_cast<size_t>(half) * kHalf * kSpread, sl,
                              sizeof(unsigned long long) * static_cast<size_t>(k) * kSpread,
                              hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipEventRecord(h->chunk_ev[half], h->stream));
    q[nq++] = Chunk{half, k};
    issued += k;
    return CPMDP_OK;
  };
  // Wait for the oldest chunk in flight; its first and last residuals.
  double rf = INFINITY, rl = INFINITY;
  int kprev = 0;
  auto collect = [&]() -> int {
    const Chunk c = q[0];
    q[0] = q[1];
    --nq;
    HIP_TRY(h, hipEventSynchronize(h->chunk_ev[c.half]));
    const unsigned long long* hs = h->host_slots + static_cast<size_t>(c.half) * kHalf * kSpread;
    for (int j = 0; j < c.k; ++j) {
      unsigned long long m = 0;
      for (int w = 0; w < kSpread; ++w) m = std::max(m, hs[static_cast<size_t>(j) * kSpread + w]);
      const double r = bits_to_double(m);
      if (!std::isfinite(r))
        return fail(h, CPMDP_E_NONFINITE, "non-finite value produced during sweeps");
      if (j == 0) rf = r;
      if (j == c.k - 1) rl = r;
    }
    *sweeps += c.k;
    kprev = c.k;
    *last_res = rl;
    return CPMDP_OK;
  };
  auto drain = [&]() -> int {
    while (nq > 0) {
      const int rc = collect();
      if (rc) return rc;
    }
    return CPMDP_OK;
  };
  int rc = CPMDP_OK;
  auto keep_trend = [&]() {
    if (trend && kprev > 0) *trend = SweepTrend{rf, rl, kprev};
  };
  if (trend && trend->k > 1 && std::isfinite(trend->rl) && trend->rl > tol) {
    // first chunks sized from the previous stage's contraction
    double need = predict_need(trend->rf, trend->rl, trend->k, h->gamma, tol);
    for (int c = 0; c < 2 && need > 0 && issued < budget && !rc; ++c) {
      const int64_t k = static_cast<int64_t>(std::min(std::max(need, 4.0), 128.0));
      rc = issue(static_cast<int>(std::min<int64_t>(k, budget - issued)));
      need -= static_cast<double>(k);
    }
  } else {
    if (issued < budget) rc = issue(static_cast<int>(std::min<int64_t>(4, budget - issued)));
    if (!rc && issued < budget) rc = issue(static_cast<int>(std::min<int64_t>(8, budget - issued)));
  }
  while (!rc && nq > 0) {
    rc = collect();
    if (rc) break;
    const bool stalled = stall_floor > 0 && rl <= stall_floor && kprev >= 8 &&
                         rl >= rf * std::max(0.9, std::pow(h->gamma, 0.5 * (kprev - 1)));
    if (rl <= tol || stalled) {
      rc = drain();
      if (rc) break;
      keep_trend();
      if (rl <= tol) {
        *done = true;
        return CPMDP_OK;
      }
      if (stalled) return CPMDP_OK;
    }
    // queue the next chunk (4..128 sweeps, bounded to keep the overshoot
    // past tol small) unless the one in flight is predicted to finish
    int64_t inflight = 0;
    for (int i = 0; i < nq; ++i) inflight += q[i].k;
    if (issued < budget) {
      const double need = predict_need(rf, rl, kprev, h->gamma, tol) - static_cast<double>(inflight);
      if (need > 0 || nq == 0) {
        const int64_t k = static_cast<int64_t>(std::min(std::max(need, 4.0), 128.0));
        rc = issue(static_cast<int>(std::min<int64_t>(k, budget - issued)));
      }
    }
  }
  if (rc) {
    (void)hipStreamSynchronize(h->stream);   // leave no chunk running on error
    return rc;
  }
  keep_trend();
  return CPMDP_OK;
}

// ||v||_inf of an FP32 vector (keys of max v and max -v, read on the host).
static int maxabs_f32(cpmdp_t* h, const float* v, double* out) {
  const hipStream_t st = h->stream;
  launch_fill_u64(h->d.vmax + 4, 2, 0ull, st);
  launch_minmax_keys_f32(v, h->S, h->d.vmax + 4, st);
  HIP_TRY(h, hipMemcpyAsync(h->host_slots, h->d.vmax + 4, 16, hipMemcpyDeviceToHost, st));
  HIP_TRY(h, hipStreamSynchronize(st));
  auto undo = [](unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return bits_to_double(b);
  };
  *out = std::max(std::fabs(undo(h->host_slots[0])), std::fabs(undo(h->host_slots[1])));
  if (!std::isfinite(*out)) return fail(h, CPMDP_E_NONFINITE, "non-finite value during sweeps");
  return CPMDP_OK;
}

// Greedy / certificate pass in FP64 over V: residual ||BV - V|| and policy.
static int certify(cpmdp_t* h, const double* V, int32_t* pi_out, const int32_t* pi_in,
                   double* res, unsigned* changes) {
  zero_slots(h, 1);
  launch_fill_u64(h->d.vmax, 1, 0ull, h->stream);
  launch_fill_u32(h->d.counters, 2, 0u, h->stream);
  launch_maxabs_f64(V, h->S, h->d.vmax, h->stream);
  sweep(h, true, MODE_GREEDY, V, nullptr, h->d.R64, pi_in, pi_out ? pi_out : h->d.piA,
        nullptr, h->d.slots, h->d.counters, false);
  int rc = check_device(h);
  if (rc) return rc;
  std::vector<double> r;
  unsigned c = 0;
  rc = read_slots(h, 1, r, &c);
  if (rc) return rc;
  *res = r[0];
  if (changes) *changes = c;
  if (!std::isfinite(*res)) return fail(h, CPMDP_E_NONFINITE, "non-finite Bellman residual");
  return CPMDP_OK;
}

// Axis structure of the stencil weights: A == 2n and action a = 2k + d
// differs from a shared vector wbase (per point, the value most actions have)
// only at the centre and its two axis-k points.  Stores the kernel-argument
// copy [wbase (2n+1) | per action: diff at centre, +e_k, -e_k].
void split_axis_weights(cpmdp_t* h) {
  const int P = 2 * h->n + 1, A = h->A;
  std::vector<double> wbase(P, 0.0), wdiff(static_cast<size_t>(A) * P, 0.0);
  for (int p = 0; p < P; ++p) {
    int best_count = 0;
    for (int a = 0; a < A; ++a) {
      int cnt = 0;
      for (int b = 0; b < A; ++b) cnt += h->w[b * P + p] == h->w[a * P + p];
      if (cnt > best_count) {
        best_count = cnt;
        wbase[p] = h->w[a * P + p];
      }
    }
    for (int a = 0; a < A; ++a) wdiff[a * P + p] = h->w[a * P + p] - wbase[p];
  }
  bool axis = (A == 2 * h->n);
  for (int a = 0; a < A && axis; ++a)
    for (int p = 0; p < P; ++p) {
      const int k = a / 2;
      if (p != 0 && p != 1 + 2 * k && p != 2 + 2 * k && wdiff[a * P + p] != 0.0) axis = false;
    }
  h->st_axis = axis ? 1 : 0;
  h->kw64.clear();
  if (axis) {
    for (int p = 0; p < P; ++p) h->kw64.push_back(wbase[p]);
    for (int a = 0; a < A; ++a) {
      const int k = a / 2;
      h->kw64.push_back(wdiff[a * P]);
      h->kw64.push_back(wdiff[a * P + 1 + 2 * k]);
      h->kw64.push_back(wdiff[a * P + 2 + 2 * k]);
    }
  }
  h->kw32.assign(h->kw64.begin(), h->kw64.end());
}

// ------------------------------------------------- Tensor-Train / Tucker

constexpr int kTTMaxBond = 8;
constexpr int kTTMaxMode = 16;

// Checks shared by the Tensor-Train and Tucker create calls.
static int check_grid_args(int32_t n_dims, const int64_t* sizes, int32_t n_actions,
                           const double* rewards, double gamma, int64_t* S_out) {
  if (!sizes || !rewards) return fail(nullptr, CPMDP_E_ARG, "NULL input array");
  if (n_dims < 1 || n_dims > kMaxDims) return fail(nullptr, CPMDP_E_ARG, "n_dims must be in [1, 8]");
  if (n_actions < 1 || n_actions > kMaxActions)
    return fail(nullptr, CPMDP_E_ARG, "n_actions must be in [1, 255]");
  int64_t S = 1;
  for (int k = 0; k < n_dims; ++k) {
    if (sizes[k] < 1) return fail(nullptr, CPMDP_E_ARG, "sizes must be >= 1");
    if (sizes[k] > kTTMaxMode)
      return fail(nullptr, CPMDP_E_UNSUPPORTED, "Tensor-Train / Tucker models need every m_k <= 16");
    S *= sizes[k];
    if (S >= (int64_t(1) << 31)) return fail(nullptr, CPMDP_E_ARG, "state count must be < 2^31");
  }
  if (!std::isfinite(gamma)) return fail(nullptr, CPMDP_E_NONFINITE, "gamma is not finite");
  if (gamma < 0.0 || gamma >= 1.0) return fail(nullptr, CPMDP_E_ARG, "gamma must be in [0, 1)");
  for (int64_t s = 0; s < S; ++s)
    if (!std::isfinite(rewards[s])) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite reward");
  *S_out = S;
  return CPMDP_OK;
}

// Validates Tensor-Train bonds [A][n+1] and cores (C ABI layout) and
// builds the handle: row sums of every P_a from the cores (the bond
// matrices M_k(i) = sum_j G_k[:, i, j, :] multiplied from the last dim, one
// vector per state), then the padded device layout of tt.hip.
static int create_tt_impl(cpmdp_t** out, int32_t n, const int64_t* sizes, int32_t A,
                          const int32_t* bonds, const double* cores, const double* rewards,
                          double gamma, int64_t S) {
  for (int a = 0; a < A; ++a) {
    const int32_t* b = bonds + static_cast<size_t>(a) * (n + 1);
    if (b[0] != 1 || b[n] != 1) return fail(nullptr, CPMDP_E_ARG, "bonds[a][0] and bonds[a][n] must be 1");
    for (int k = 0; k <= n; ++k) {
      if (b[k] < 1) return fail(nullptr, CPMDP_E_ARG, "bonds must be >= 1");
      if (b[k] > kTTMaxBond) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "bond %d of action %d is %d; at most %d is supported", k, a,
                      b[k], kTTMaxBond);
        return fail(nullptr, CPMDP_E_UNSUPPORTED, buf);
      }
    }
  }
  std::vector<int64_t> off(static_cast<size_t>(A) * n);
  int64_t count = 0;
  for (int a = 0; a < A; ++a)
    for (int k = 0; k < n; ++k) {
      off[static_cast<size_t>(a) * n + k] = count;
      count += static_cast<int64_t>(bonds[a * (n + 1) + k]) * sizes[k] * sizes[k] *
               bonds[a * (n + 1) + k + 1];
    }
  for (int64_t i = 0; i < count; ++i) {
    if (!std::isfinite(cores[i])) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite core entry");
    if (cores[i] < 0.0) return fail(nullptr, CPMDP_E_NOT_STOCHASTIC, "negative core entry");
  }
  for (int a = 0; a < A; ++a) {
    // w[(rest) * br + r]: row sums of the trailing dims' operator with open bond r
    std::vector<double> w(1, 1.0), nw;
    int64_t rest = 1;
    for (int k = n - 1; k >= 0; --k) {
      const int64_t m = sizes[k];
      const int bl = bonds[a * (n + 1) + k], br = bonds[a * (n + 1) + k + 1];
      const double* G = cores + off[static_cast<size_t>(a) * n + k];
      std::vector<double> M(static_cast<size_t>(bl) * m * br, 0.0);   // [l][i][r]
      for (int l = 0; l < bl; ++l)
        for (int64_t i = 0; i < m; ++i)
          for (int64_t j = 0; j < m; ++j)
            for (int r = 0; r < br; ++r)
              M[(l * m + i) * br + r] += G[((l * m + i) * m + j) * br + r];
      nw.assign(static_cast<size_t>(m * rest * bl), 0.0);
      for (int64_t i = 0; i < m; ++i)
        for (int64_t q = 0; q < rest; ++q)
          for (int l = 0; l < bl; ++l) {
            double acc = 0.0;
            for (int r = 0; r < br; ++r) acc += M[(l * m + i) * br + r] * w[q * br + r];
            nw[(i * rest + q) * bl + l] = acc;
          }
      w.swap(nw);
      rest *= m;
    }
    for (int64_t s = 0; s < S; ++s)
      if (std::fabs(w[s] - 1.0) > 1e-9) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "row %lld of the operator of action %d sums to %.17g",
                      (long long)s, a, w[s]);
        return fail(nullptr, CPMDP_E_NOT_STOCHASTIC, buf);
      }
  }
  cpmdp_t* h = new (std::nothrow) cpmdp_t();
  if (!h) return fail(nullptr, CPMDP_E_ARG, "out of host memory");
  h->n = n;
  h->S = S;
  h->A = A;
  h->gamma = gamma;
  h->sizes.assign(sizes, sizes + n);
  h->rewards.assign(rewards, rewards + S);
  for (int64_t s = 0; s < S; ++s) h->rmax = std::max(h->rmax, std::fabs(rewards[s]));
  h->terminal.assign(static_cast<size_t>(S), 0);
  h->path = CPMDP_PATH_TT;
  h->geom = make_geom(h);
  h->t_bonds.assign(bonds, bonds + static_cast<size_t>(A) * (n + 1));
  h->t_mm.resize(n);
  for (int k = 0; k < n; ++k) h->t_mm[k] = sizes[k] <= 4 ? 4 : (sizes[k] <= 8 ? 8 : 16);
  h->t_maxb = 1;
  for (int32_t b : h->t_bonds) h->t_maxb = std::max(h->t_maxb, b);
  // padded device layout Gd[r][j][l][i] per (action, dim)
  h->t_off.resize(static_cast<size_t>(A) * n);
  int64_t dcount = 0;
  for (int a = 0; a < A; ++a)
    for (int k = 0; k < n; ++k) {
      const int64_t mm = h->t_mm[k];
      const int64_t lp = (bonds[a * (n + 1) + k] + 3) & ~3;
      h->t_off[static_cast<size_t>(a) * n + k] = dcount;
      dcount += bonds[a * (n + 1) + k + 1] * mm * lp * mm;
    }
  h->t_core.assign(static_cast<size_t>(dcount), 0.0);
  for (int a = 0; a < A; ++a)
    for (int k = 0; k < n; ++k) {
      const int64_t m = sizes[k], mm = h->t_mm[k];
      const int bl = bonds[a * (n + 1) + k], br = bonds[a * (n + 1) + k + 1];
      const int64_t lp = (bl + 3) & ~3;
      const double* G = cores + off[static_cast<size_t>(a) * n + k];
      double* D = h->t_core.data() + h->t_off[static_cast<size_t>(a) * n + k];
      for (int l = 0; l < bl; ++l)
        for (int64_t i = 0; i < m; ++i)
          for (int64_t j = 0; j < m; ++j)
            for (int r = 0; r < br; ++r)
              D[((r * mm + j) * lp + l) * mm + i] = G[((l * m + i) * m + j) * br + r];
    }
  *out = h;
  return CPMDP_OK;
}

}  // namespace cpm

using namespace cpm;

// =================================================================== C ABI

extern "C" {

int cpmdp_create(cpmdp_t** out, int32_t n_dims, const int64_t* sizes, int32_t n_actions,
                 const int32_t* ranks, const double* factors, const double* lambdas,
                 const double* rewards, double gamma) {
  if (!out) return fail(nullptr, CPMDP_E_ARG, "out is NULL");
  *out = nullptr;
  if (!sizes || !ranks || !factors || !lambdas || !rewards)
    return fail(nullptr, CPMDP_E_ARG, "NULL input array");
  if (n_dims < 1 || n_dims > kMaxDims) return fail(nullptr, CPMDP_E_ARG, "n_dims must be in [1, 8]");
  if (n_actions < 1 || n_actions > kMaxActions)
    return fail(nullptr, CPMDP_E_ARG, "n_actions must be in [1, 255]");
  int64_t S = 1;
  for (int k = 0; k < n_dims; ++k) {
    if (sizes[k] < 1) return fail(nullptr, CPMDP_E_ARG, "sizes must be >= 1");
    if (sizes[k] > (1 << 30)) return fail(nullptr, CPMDP_E_ARG, "size too large");
    S *= sizes[k];
    if (S >= (int64_t(1) << 31)) return fail(nullptr, CPMDP_E_ARG, "state count must be < 2^31");
  }
  int64_t T = 0;
  for (int a = 0; a < n_actions; ++a) {
    if (ranks[a] < 1) return fail(nullptr, CPMDP_E_ARG, "ranks must be >= 1");
    T += ranks[a];
  }
  if (T > (1 << 20)) return fail(nullptr, CPMDP_E_ARG, "too many rank terms");
  if (!std::isfinite(gamma)) return fail(nullptr, CPMDP_E_NONFINITE, "gamma is not finite");
  if (gamma < 0.0 || gamma >= 1.0) return fail(nullptr, CPMDP_E_ARG, "gamma must be in [0, 1)");
  int64_t term_stride = 0;
  for (int k = 0; k < n_dims; ++k) term_stride += sizes[k] * sizes[k];
  const int64_t F = T * term_stride;
  for (int64_t i = 0; i < F; ++i)
    if (!std::isfinite(factors[i])) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite factor entry");
  for (int64_t i = 0; i < T; ++i)
    if (!std::isfinite(lambdas[i])) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite lambda");
  for (int64_t s = 0; s < S; ++s)
    if (!std::isfinite(rewards[s])) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite reward");
  // stochasticity of every factor row and of every action's lambdas
  for (int64_t t = 0; t < T; ++t) {
    int64_t off = t * term_stride;
    for (int k = 0; k < n_dims; ++k) {
      const int64_t m = sizes[k];
      for (int64_t i = 0; i < m; ++i) {
        double sum = 0.0;
        for (int64_t j = 0; j < m; ++j) {
          const double v = factors[off + i * m + j];
          if (v < 0.0) {
            char buf[160];
            std::snprintf(buf, sizeof buf, "negative probability in term %lld dim %d row %lld",
                          (long long)t, k, (long long)i);
            return fail(nullptr, CPMDP_E_NOT_STOCHASTIC, buf);
          }
          sum += v;
        }
        if (std::fabs(sum - 1.0) > 1e-12) {
          char buf[160];
          std::snprintf(buf, sizeof buf, "row %lld of factor (term %lld, dim %d) sums to %.17g",
                        (long long)i, (long long)t, k, sum);
          return fail(nullptr, CPMDP_E_NOT_STOCHASTIC, buf);
        }
      }
      off += m * m;
    }
  }
  {
    int64_t t = 0;
    for (int a = 0; a < n_actions; ++a) {
      double sum = 0.0;
      for (int r = 0; r < ranks[a]; ++r, ++t) {
        if (lambdas[t] < 0.0) return fail(nullptr, CPMDP_E_NOT_STOCHASTIC, "negative lambda");
        sum += lambdas[t];
      }
      if (std::fabs(sum - 1.0) > 1e-12) {
        char buf[128];
        std::snprintf(buf, sizeof buf, "lambdas of action %d sum to %.17g", a, sum);
        return fail(nullptr, CPMDP_E_NOT_STOCHASTIC, buf);
      }
    }
  }

  cpmdp_t* h = new (std::nothrow) cpmdp_t();
  if (!h) return fail(nullptr, CPMDP_E_ARG, "out of host memory");
  h->n = n_dims;
  h->S = S;
  h->A = n_actions;
  h->gamma = gamma;
  h->sizes.assign(sizes, sizes + n_dims);
  h->ranks.assign(ranks, ranks + n_actions);
  h->factors.assign(factors, factors + F);
  h->lambdas.assign(lambdas, lambdas + T);
  h->rewards.assign(rewards, rewards + S);
  for (int64_t s = 0; s < S; ++s) h->rmax = std::max(h->rmax, std::fabs(rewards[s]));
  h->terminal.assign(static_cast<size_t>(S), 0);
  h->term_start.resize(n_actions + 1);
  h->term_start[0] = 0;
  for (int a = 0; a < n_actions; ++a) h->term_start[a + 1] = h->term_start[a] + ranks[a];
  h->kinds.resize(static_cast<size_t>(T) * n_dims);
  bool stencil = true;
  for (int64_t t = 0; t < T; ++t) {
    int64_t off = t * term_stride;
    int non_id = 0;
    for (int k = 0; k < n_dims; ++k) {
      const int kind = classify(factors + off, static_cast<int>(sizes[k]));
      h->kinds[t * n_dims + k] = static_cast<uint8_t>(kind);
      if (kind != F_IDENT) ++non_id;
      if (kind == F_DENSE) stencil = false;
      off += sizes[k] * sizes[k];
    }
    if (non_id > 1) stencil = false;
  }
  h->path = stencil ? CPMDP_PATH_STENCIL : CPMDP_PATH_DENSE;
  h->geom = make_geom(h);
  {
    // persistent stencil grid: contiguous ranges of whole 256 x vec chunks
    h->st_vec = (sizes[n_dims - 1] % 4 == 0) ? 4 : 1;
    const int64_t chunk = static_cast<int64_t>(kBlock) * h->st_vec;
    const int64_t units = (S + chunk - 1) / chunk;
    int64_t nb = std::min<int64_t>(units, kMaxBlocks);
    const int64_t per = (units + nb - 1) / nb;
    h->st_states_per_block = static_cast<int32_t>(per * chunk);
    h->st_blocks = static_cast<int32_t>((units + per - 1) / per);
    // marching form when the planes of fixed i_0 are large (the dim-0
    // neighbours then sit far apart in memory) and there are enough planes
    const int64_t plane = S / sizes[0];
    if (n_dims >= 2 && h->st_vec == 4 && plane >= kMarchMinPlane && sizes[0] >= 8) {
      const int64_t tiles = (plane + 4 * kBlock - 1) / (4 * kBlock);
      const int64_t nseg = std::max<int64_t>(1, std::min<int64_t>(kMaxBlocks / tiles, sizes[0] / 8));
      const int64_t seg = (sizes[0] + nseg - 1) / nseg;
      h->st_march = 1;
      h->st_march_tiles = static_cast<int32_t>(tiles);
      h->st_march_seg = static_cast<int32_t>(seg);
      h->st_march_blocks = static_cast<int32_t>(tiles * ((sizes[0] + seg - 1) / seg));
    }
  }
  if (stencil) {
    const int P = 2 * n_dims + 1;
    h->w.assign(static_cast<size_t>(n_actions) * P, 0.0);
    for (int a = 0; a < n_actions; ++a)
      for (int t = h->term_start[a]; t < h->term_start[a + 1]; ++t) {
        int p = 0;
        for (int k = 0; k < n_dims; ++k) {
          const int kind = h->kinds[t * n_dims + k];
          if (kind == F_SHIFT_P) p = 1 + 2 * k;
          if (kind == F_SHIFT_M) p = 2 + 2 * k;
        }
        h->w[a * P + p] += lambdas[t];
      }
    split_axis_weights(h);
  } else {
    if (!choose_split(h->sizes, S, sizeof(double), h->cg64) ||
        !choose_split(h->sizes, S, sizeof(float), h->cg32)) {
      delete h;
      return fail(nullptr, CPMDP_E_UNSUPPORTED,
                  "dense factors need every m_k <= 32 and a row/column split of the "
                  "dimensions that fits LDS");
    }
  }
  *out = h;
  return CPMDP_OK;
}

int cpmdp_create_lists(cpmdp_t** out, int64_t n_states, int32_t n_actions,
                       const int64_t* row_ptr, const int64_t* succ, const double* prob,
                       const double* rewards, double gamma) {
  if (!out) return fail(nullptr, CPMDP_E_ARG, "out is NULL");
  *out = nullptr;
  if (!row_ptr || !rewards) return fail(nullptr, CPMDP_E_ARG, "NULL input array");
  if (n_states < 1 || n_states > (int64_t{1} << 30))
    return fail(nullptr, CPMDP_E_ARG, "n_states must be in [1, 2^30]");
  if (n_actions < 1 || n_actions > kMaxActions)
    return fail(nullptr, CPMDP_E_ARG, "n_actions must be in [1, 255]");
  if (!std::isfinite(gamma)) return fail(nullptr, CPMDP_E_NONFINITE, "gamma is not finite");
  if (!(gamma >= 0.0 && gamma < 1.0)) return fail(nullptr, CPMDP_E_ARG, "gamma must be in [0, 1)");
  const int64_t S = n_states, A = n_actions, rows = S * A;
  if (row_ptr[0] != 0) return fail(nullptr, CPMDP_E_ARG, "row_ptr[0] must be 0");
  for (int64_t r = 0; r < rows; ++r)
    if (row_ptr[r + 1] < row_ptr[r]) return fail(nullptr, CPMDP_E_ARG, "row_ptr must not decrease");
  const int64_t nnz = row_ptr[rows];
  if (nnz > 0 && (!succ || !prob)) return fail(nullptr, CPMDP_E_ARG, "NULL succ / prob");
  for (int64_t s = 0; s < S; ++s)
    if (!std::isfinite(rewards[s])) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite reward");
  for (int64_t r = 0; r < rows; ++r) {
    double sum = 0.0;
    for (int64_t e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
      if (succ[e] < 0 || succ[e] >= S) return fail(nullptr, CPMDP_E_ARG, "successor out of range");
      if (!std::isfinite(prob[e])) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite probability");
      if (prob[e] < 0.0) return fail(nullptr, CPMDP_E_NOT_STOCHASTIC, "negative probability");
      sum += prob[e];
    }
    if (std::fabs(sum - 1.0) > 1e-9) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "list of action %lld, state %lld sums to %.17g",
                    (long long)(r / S), (long long)(r % S), sum);
      return fail(nullptr, CPMDP_E_NOT_STOCHASTIC, buf);
    }
  }
  cpmdp_t* h = new (std::nothrow) cpmdp_t();
  if (!h) return fail(nullptr, CPMDP_E_ARG, "out of host memory");
  h->n = 1;
  h->S = S;
  h->A = n_actions;
  h->gamma = gamma;
  h->sizes.assign(1, S);
  h->rewards.assign(rewards, rewards + S);
  for (int64_t s = 0; s < S; ++s) h->rmax = std::max(h->rmax, std::fabs(rewards[s]));
  h->terminal.assign(static_cast<size_t>(S), 0);
  h->path = CPMDP_PATH_LISTS;
  // Sliced layout: per 64-state slice and action, as many columns as the
  // slice's longest list; entry of lane l in column c at c * 64 + l.
  const int64_t nsl = (S + kSlice - 1) / kSlice;
  h->l_nslices = static_cast<int32_t>(nsl);
  h->l_cols.assign(static_cast<size_t>(nsl * A + 1), 0);
  int64_t cols = 0;
  for (int64_t q = 0; q < nsl; ++q)
    for (int64_t a = 0; a < A; ++a) {
      int64_t w = 0;
      for (int64_t s = q * kSlice; s < std::min(S, (q + 1) * kSlice); ++s)
        w = std::max(w, row_ptr[a * S + s + 1] - row_ptr[a * S + s]);
      cols += w;
      if (cols * kSlice >= (int64_t{1} << 31)) {
        delete h;
        return fail(nullptr, CPMDP_E_UNSUPPORTED, "successor lists too long (2^31 padded entries)");
      }
      h->l_cols[q * A + a + 1] = static_cast<int32_t>(cols);
    }
  h->l_succ.assign(static_cast<size_t>(cols * kSlice), 0);
  h->l_prob.assign(static_cast<size_t>(cols * kSlice), 0.0);
  for (int64_t q = 0; q < nsl; ++q)
    for (int64_t a = 0; a < A; ++a) {
      const int64_t c0 = h->l_cols[q * A + a];
      const int64_t w = h->l_cols[q * A + a + 1] - c0;
      for (int64_t l = 0; l < kSlice; ++l) {
        const int64_t s = q * kSlice + l;
        const int64_t r0 = s < S ? row_ptr[a * S + s] : 0, len = s < S ? row_ptr[a * S + s + 1] - r0 : 0;
        for (int64_t j = 0; j < w; ++j) {
          const size_t e = static_cast<size_t>((c0 + j) * kSlice + l);
          if (j < len) {
            h->l_succ[e] = static_cast<int32_t>(succ[r0 + j]);
            h->l_prob[e] = prob[r0 + j];
          } else {
            h->l_succ[e] = static_cast<int32_t>(s < S ? s : 0);   // padding: weight 0
          }
        }
      }
    }
  // blocks of 4 waves, each block a contiguous range of slices
  const int64_t units = (nsl + kBlock / kSlice - 1) / (kBlock / kSlice);
  const int64_t nb = std::min<int64_t>(units, kMaxBlocks);
  const int64_t per_units = (units + nb - 1) / nb;
  h->l_slices_per_block = static_cast<int32_t>(per_units * (kBlock / kSlice));
  h->l_blocks = static_cast<int32_t>((nsl + h->l_slices_per_block - 1) / h->l_slices_per_block);
  *out = h;
  return CPMDP_OK;
}

int cpmdp_create_tt(cpmdp_t** out, int32_t n_dims, const int64_t* sizes, int32_t n_actions,
                    const int32_t* bonds, const double* cores, const double* rewards,
                    double gamma) {
  if (!out) return fail(nullptr, CPMDP_E_ARG, "out is NULL");
  *out = nullptr;
  if (!bonds || !cores) return fail(nullptr, CPMDP_E_ARG, "NULL input array");
  int64_t S = 0;
  const int rc = check_grid_args(n_dims, sizes, n_actions, rewards, gamma, &S);
  if (rc) return rc;
  return create_tt_impl(out, n_dims, sizes, n_actions, bonds, cores, rewards, gamma, S);
}

int cpmdp_create_tucker(cpmdp_t** out, int32_t n_dims, const int64_t* sizes, int32_t n_actions,
                        const int32_t* core_ranks, const double* cores, const double* factors,
                        const double* rewards, double gamma) {
  if (!out) return fail(nullptr, CPMDP_E_ARG, "out is NULL");
  *out = nullptr;
  if (!core_ranks || !cores || !factors) return fail(nullptr, CPMDP_E_ARG, "NULL input array");
  int64_t S = 0;
  int rc = check_grid_args(n_dims, sizes, n_actions, rewards, gamma, &S);
  if (rc) return rc;
  const int n = n_dims, A = n_actions;
  int64_t ccount = 0, fcount = 0;
  for (int a = 0; a < A; ++a) {
    int64_t c = 1;
    for (int k = 0; k < n; ++k) {
      const int32_t R = core_ranks[a * n + k];
      if (R < 1) return fail(nullptr, CPMDP_E_ARG, "core ranks must be >= 1");
      if (R > kTTMaxBond) return fail(nullptr, CPMDP_E_UNSUPPORTED, "core ranks must be <= 8");
      c *= R;
      fcount += R * sizes[k] * sizes[k];
    }
    ccount += c;
  }
  for (int64_t i = 0; i < ccount; ++i) {
    if (!std::isfinite(cores[i])) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite core entry");
    if (cores[i] < 0.0) return fail(nullptr, CPMDP_E_NOT_STOCHASTIC, "negative core entry");
  }
  for (int64_t i = 0; i < fcount; ++i) {
    if (!std::isfinite(factors[i])) return fail(nullptr, CPMDP_E_NONFINITE, "non-finite factor entry");
    if (factors[i] < 0.0) return fail(nullptr, CPMDP_E_NOT_STOCHASTIC, "negative probability");
  }
  // Rewrite each action as a Tensor-Train, splitting at dim mu: the bond
  // left of dim k <= mu carries (r_0..r_{k-1}), the bond left of dim k > mu
  // carries (r_k..r_{n-1}); core mu contracts the Tucker core:
  //   k < mu : G_k[(r_<k), i, j, (r_<k, r_k)]   = U^(k)_{r_k}[i, j]
  //   k = mu : G_mu[(r_<mu), i, j, (r_>mu)]     = sum_{r_mu} C[r] U^(mu)_{r_mu}[i, j]
  //   k > mu : G_k[(r_k, r_>k), i, j, (r_>k)]   = U^(k)_{r_k}[i, j]
  // so the bond products enforce equal indices and sum C[r] kron_k U.  mu
  // minimises the largest bond (then the flop count of a sweep).
  std::vector<int32_t> bonds(static_cast<size_t>(A) * (n + 1));
  std::vector<double> tt;
  const double* C = cores;
  const double* U = factors;
  for (int a = 0; a < A; ++a) {
    const int32_t* R = core_ranks + static_cast<size_t>(a) * n;
    int best_mu = 0;
    int64_t best_max = INT64_MAX, best_cost = INT64_MAX;
    std::vector<int64_t> bb(n + 1);
    for (int mu = 0; mu < n; ++mu) {
      bb[0] = bb[n] = 1;
      for (int k = 1; k < n; ++k) {
        int64_t p = 1;
        if (k <= mu) for (int l = 0; l < k; ++l) p *= R[l];
        else for (int l = k; l < n; ++l) p *= R[l];
        bb[k] = p;
      }
      int64_t mx = 0, cost = 0;
      for (int k = 0; k <= n; ++k) mx = std::max(mx, bb[k]);
      for (int k = 0; k < n; ++k) cost += bb[k] * bb[k + 1] * sizes[k];
      if (mx < best_max || (mx == best_max && cost < best_cost)) {
        best_mu = mu;
        best_max = mx;
        best_cost = cost;
      }
    }
    const int mu = best_mu;
    if (best_max > kTTMaxBond) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "the core of action %d needs a Tensor-Train bond of %lld; "
                    "at most %d is supported", a, (long long)best_max, kTTMaxBond);
      return fail(nullptr, CPMDP_E_UNSUPPORTED, buf);
    }
    std::vector<int64_t> pre(n + 1, 1), suf(n + 1, 1);   // prod R[0..k), prod R[k..n)
    for (int k = 0; k < n; ++k) pre[k + 1] = pre[k] * R[k];
    for (int k = n - 1; k >= 0; --k) suf[k] = suf[k + 1] * R[k];
    int32_t* b = bonds.data() + static_cast<size_t>(a) * (n + 1);
    for (int k = 0; k <= n; ++k)
      b[k] = static_cast<int32_t>(k == 0 || k == n ? 1 : (k <= mu ? pre[k] : suf[k]));
    std::vector<const double*> Uk(n);   // factor blocks of action a, dim k
    {
      const double* u = U;
      for (int k = 0; k < n; ++k) {
        Uk[k] = u;
        u += R[k] * sizes[k] * sizes[k];
      }
      U = u;
    }
    for (int k = 0; k < n; ++k) {
      const int64_t m = sizes[k];
      const int64_t bl = b[k], br = b[k + 1];
      const size_t base = tt.size();
      tt.resize(base + static_cast<size_t>(bl * m * m * br), 0.0);
      double* G = tt.data() + base;
      auto at = [&](int64_t l, int64_t i, int64_t j, int64_t r) -> double& {
        return G[((l * m + i) * m + j) * br + r];
      };
      if (k < mu) {
        for (int64_t l = 0; l < bl; ++l)
          for (int64_t rk = 0; rk < R[k]; ++rk)
            for (int64_t i = 0; i < m; ++i)
              for (int64_t j = 0; j < m; ++j) at(l, i, j, l * R[k] + rk) = Uk[k][(rk * m + i) * m + j];
      } else if (k > mu) {
        for (int64_t rk = 0; rk < R[k]; ++rk)
          for (int64_t r = 0; r < br; ++r)
            for (int64_t i = 0; i < m; ++i)
              for (int64_t j = 0; j < m; ++j) at(rk * br + r, i, j, r) = Uk[k][(rk * m + i) * m + j];
      } else {
        for (int64_t l = 0; l < bl; ++l)
          for (int64_t rk = 0; rk < R[k]; ++rk)
            for (int64_t r = 0; r < br; ++r) {
              const double cw = C[(l * R[k] + rk) * br + r];
              for (int64_t i = 0; i < m; ++i)
                for (int64_t j = 0; j < m; ++j) at(l, i, j, r) += cw * Uk[k][(rk * m + i) * m + j];
            }
      }
    }
    C += pre[n];
  }
  return create_tt_impl(out, n, sizes, A, bonds.data(), tt.data(), rewards, gamma, S);
}

int cpmdp_set_terminal(cpmdp_t* h, const uint8_t* mask) {
  if (!h) return fail(nullptr, CPMDP_E_ARG, "handle is NULL");
  if (!mask) return fail(h, CPMDP_E_ARG, "mask is NULL");
  if (h->bound) return fail(h, CPMDP_E_STATE, "set_terminal must precede bind");
  for (int64_t s = 0; s < h->S; ++s) h->terminal[s] = mask[s] ? 1 : 0;
  return CPMDP_OK;
}

int cpmdp_set_obstacles(cpmdp_t* h, const uint8_t* mask) {
  if (!h) return fail(nullptr, CPMDP_E_ARG, "handle is NULL");
  if (!mask) return fail(h, CPMDP_E_ARG, "mask is NULL");
  if (h->bound) return fail(h, CPMDP_E_STATE, "set_obstacles must precede bind");
  bool any = false;
  for (int64_t s = 0; s < h->S && !any; ++s) any = mask[s] != 0;
  if (!any) {
    h->obstacle.clear();
    return CPMDP_OK;
  }
  if (h->path != CPMDP_PATH_STENCIL)
    return fail(h, CPMDP_E_UNSUPPORTED,
                "obstacles need shift/identity factors: with dense factors or Tensor-Train / "
                "Tucker cores the blocked moves are not a sparse correction of the operator, "
                "and successor lists encode blocked moves themselves");
  h->obstacle.assign(static_cast<size_t>(h->S), 0);
  for (int64_t s = 0; s < h->S; ++s) h->obstacle[s] = mask[s] ? 1 : 0;
  return CPMDP_OK;
}

int cpmdp_get_path(const cpmdp_t* h, int32_t* path) {
  if (!h || !path) return fail(nullptr, CPMDP_E_ARG, "NULL argument");
  *path = h->path;
  return CPMDP_OK;
}

int cpmdp_workspace_bytes(const cpmdp_t* h, size_t* bytes) {
  if (!h || !bytes) return fail(nullptr, CPMDP_E_ARG, "NULL argument");
  DevPtrs tmp;
  layout(h, &tmp, nullptr, bytes);
  return CPMDP_OK;
}

int cpmdp_set_option(cpmdp_t* h, int option, int64_t value) {
  if (!h) return fail(nullptr, CPMDP_E_ARG, "handle is NULL");
  if (option == CPMDP_OPT_MARCH) {
    if (value != 0 && value != 1) return fail(h, CPMDP_E_ARG, "option value must be 0 or 1");
    h->opt_march = value != 0;
    return CPMDP_OK;
  }
  return fail(h, CPMDP_E_ARG, "unknown option");
}

int cpmdp_bind(cpmdp_t* h, void* ws, size_t bytes, void* stream) {
  if (!h) return fail(nullptr, CPMDP_E_ARG, "handle is NULL");
  if (!ws) return fail(h, CPMDP_E_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
    return fail(h, CPMDP_E_WORKSPACE, "workspace must be 256-byte aligned");
  size_t need = 0;
  DevPtrs tmp;
  layout(h, &tmp, nullptr, &need);
  if (bytes < need) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "workspace has %zu bytes, %zu needed", bytes, need);
    return fail(h, CPMDP_E_WORKSPACE, buf);
  }
  h->stream = static_cast<hipStream_t>(stream);
  if (h->path == CPMDP_PATH_DENSE) {
    int dev = 0, lds = 0;
    HIP_TRY(h, hipGetDevice(&dev));
    HIP_TRY(h, hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const int64_t need_lds = std::max(chain_lds_bytes(h->cg64, 8), chain_lds_bytes(h->cg32, 4));
    if (need_lds > lds) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "chain kernels need %lld bytes of LDS per block, device has %d",
                    (long long)need_lds, lds);
      return fail(h, CPMDP_E_UNSUPPORTED, buf);
    }
  }
  layout(h, &h->d, static_cast<char*>(ws), &need);
  h->ws = static_cast<char*>(ws);
  h->ws_bytes = bytes;
  if (!h->host_slots) {
    HIP_TRY(h, hipHostMalloc(reinterpret_cast<void**>(&h->host_slots),
                             sizeof(unsigned long long) * kSlots * kSpread,
                             hipHostMallocDefault));
    HIP_TRY(h, hipHostMalloc(reinterpret_cast<void**>(&h->host_ctr), sizeof(unsigned) * 8,
                             hipHostMallocDefault));
    for (auto& e : h->chunk_ev) HIP_TRY(h, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  const size_t S = static_cast<size_t>(h->S);
  const bool obst = !h->obstacle.empty();
  if (obst)
    for (size_t s = 0; s < S; ++s)
      if (h->obstacle[s] && h->terminal[s])
        return fail(h, CPMDP_E_ARG, "a state is both terminal and an obstacle");
  // An obstacle state is outside the problem: reward 0 and no continuation
  // (so V = 0 there); moves into it are blocked (the obs masks below).
  std::vector<double> r64(h->rewards);
  std::vector<float> f32(S);
  std::vector<uint32_t> bits((S + 31) / 32 + 1, 0u);
  for (size_t s = 0; s < S; ++s) {
    const bool ob = obst && h->obstacle[s];
    if (ob) r64[s] = 0.0;
    f32[s] = static_cast<float>(r64[s]);
    if (h->terminal[s] || ob) bits[s >> 5] |= 1u << (s & 31);
  }
  std::vector<uint16_t> blocked;
  if (obst) {
    // bit 2k (2k + 1) of state s: its +e_k (-e_k) neighbour is an obstacle
    blocked.assign(S, 0);
    for (size_t o = 0; o < S; ++o) {
      if (!h->obstacle[o]) continue;
      int64_t rem = static_cast<int64_t>(o), stride = 1;
      for (int k = h->n - 1; k >= 0; --k) {
        const int64_t i = rem % h->sizes[k];
        rem /= h->sizes[k];
        if (i > 0) blocked[o - stride] |= static_cast<uint16_t>(1u << (2 * k));
        if (i < h->sizes[k] - 1) blocked[o + stride] |= static_cast<uint16_t>(1u << (2 * k + 1));
        stride *= h->sizes[k];
      }
    }
  }
  const hipStream_t st = h->stream;
  HIP_TRY(h, hipMemcpyAsync(h->d.R64, r64.data(), S * 8, hipMemcpyHostToDevice, st));
  HIP_TRY(h, hipMemcpyAsync(h->d.R32, f32.data(), S * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(h, hipMemcpyAsync(h->d.tbits, bits.data(), bits.size() * 4, hipMemcpyHostToDevice, st));
  if (obst)
    HIP_TRY(h, hipMemcpyAsync(h->d.obs, blocked.data(), S * 2, hipMemcpyHostToDevice, st));
  std::vector<float> w32;
  std::vector<float> fac32, lam32;
  std::vector<uint16_t> facbf;
  std::vector<int32_t> ts;
  std::vector<float> lp32;
  std::vector<float> tc32;
  if (h->path == CPMDP_PATH_TT) {
    const size_t nc = h->t_core.size();
    tc32.resize(nc);
    for (size_t i = 0; i < nc; ++i) tc32[i] = static_cast<float>(h->t_core[i]);
    HIP_TRY(h, hipMemcpyAsync(h->d.t_core64, h->t_core.data(), nc * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.t_core32, tc32.data(), nc * 4, hipMemcpyHostToDevice, st));
  } else if (h->path == CPMDP_PATH_LISTS) {
    const size_t ent = h->l_succ.size();
    lp32.resize(ent);
    for (size_t i = 0; i < ent; ++i) lp32[i] = static_cast<float>(h->l_prob[i]);
    HIP_TRY(h, hipMemcpyAsync(h->d.l_cols, h->l_cols.data(), h->l_cols.size() * 4,
                              hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.l_succ, h->l_succ.data(), ent * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.l_p64, h->l_prob.data(), ent * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.l_p32, lp32.data(), ent * 4, hipMemcpyHostToDevice, st));
  } else if (h->path == CPMDP_PATH_STENCIL) {
    const int P = 2 * h->n + 1, A = h->A;
    std::vector<double> w64(3 * static_cast<size_t>(A) * P, 0.0);
    std::copy(h->w.begin(), h->w.end(), w64.begin());
    w32.resize(w64.size());
    for (size_t i = 0; i < w64.size(); ++i) w32[i] = static_cast<float>(w64[i]);
    HIP_TRY(h, hipMemcpyAsync(h->d.w64, w64.data(), w64.size() * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.w32, w32.data(), w32.size() * 4, hipMemcpyHostToDevice, st));
  } else {
    const size_t F = h->factors.size();
    fac32.resize(F);
    facbf.resize(2 * F);
    auto to_bf16 = [](float f) {          // round to nearest even
      uint32_t u;
      std::memcpy(&u, &f, 4);
      return static_cast<uint16_t>((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    };
    auto from_bf16 = [](uint16_t b) {
      const uint32_t u = static_cast<uint32_t>(b) << 16;
      float f;
      std::memcpy(&f, &u, 4);
      return f;
    };
    for (size_t i = 0; i < F; ++i) {
      const float f = static_cast<float>(h->factors[i]);
      fac32[i] = f;
      facbf[i] = to_bf16(f);                          // hi
      facbf[F + i] = to_bf16(f - from_bf16(facbf[i]));  // lo (the difference is exact)
    }
    lam32.resize(h->lambdas.size());
    for (size_t i = 0; i < lam32.size(); ++i) lam32[i] = static_cast<float>(h->lambdas[i]);
    ts.assign(h->term_start.begin(), h->term_start.end());
    HIP_TRY(h, hipMemcpyAsync(h->d.fac64, h->factors.data(), F * 8, hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.fac32, fac32.data(), F * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.facbf, facbf.data(), 2 * F * 2, hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.lam64, h->lambdas.data(), lam32.size() * 8,
                              hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.lam32, lam32.data(), lam32.size() * 4, hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.kinds, h->kinds.data(), h->kinds.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(h, hipMemcpyAsync(h->d.term_start, ts.data(), ts.size() * 4, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(h, hipStreamSynchronize(st));
  h->bound = true;
  return CPMDP_OK;
}

int cpmdp_set_stream(cpmdp_t* h, void* stream) {
  if (!h) return fail(nullptr, CPMDP_E_ARG, "handle is NULL");
  h->stream = static_cast<hipStream_t>(stream);
  return CPMDP_OK;
}

static int check_common(cpmdp_t* h, int precision) {
  if (!h) return fail(nullptr, CPMDP_E_ARG, "handle is NULL");
  if (!h->bound) return fail(h, CPMDP_E_STATE, "handle is not bound to a workspace");
  if (precision < CPMDP_FP64 || precision > CPMDP_BF16)
    return fail(h, CPMDP_E_ARG, "unknown precision");
  if (precision == CPMDP_BF16 && h->path == CPMDP_PATH_LISTS)
    return fail(h, CPMDP_E_UNSUPPORTED, "successor lists run in FP64 or FP32 (no matrix product)");
  if (precision == CPMDP_BF16 && h->path == CPMDP_PATH_TT)
    return fail(h, CPMDP_E_UNSUPPORTED, "Tensor-Train / Tucker models run in FP64 or FP32");
  return CPMDP_OK;
}

static int check_policy(cpmdp_t* h, const int32_t* pi) {
  launch_fill_u32(h->d.counters + 4, 1, 0u, h->stream);
  launch_check_policy(pi, h->S, h->A, h->d.counters + 4, h->stream);
  HIP_TRY(h, hipMemcpyAsync(h->host_ctr + 4, h->d.counters + 4, 4, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (h->host_ctr[4] != 0) return fail(h, CPMDP_E_ARG, "policy holds actions outside [0, A)");
  return CPMDP_OK;
}

int cpmdp_backup(cpmdp_t* h, const void* V_in, void* V_out, int32_t* pi_out,
                 double* residual_host, int precision) {
  int rc = check_common(h, precision);
  if (rc) return rc;
  if (!V_in || !V_out) return fail(h, CPMDP_E_ARG, "NULL value buffer");
  if (V_in == V_out) return fail(h, CPMDP_E_ARG, "V_in and V_out must not alias");
  const bool p64 = precision == CPMDP_FP64;
  zero_slots(h, 1);
  if (pi_out) {
    launch_fill_u64(h->d.vmax, 1, 0ull, h->stream);
    if (p64) {
      launch_maxabs_f64(static_cast<const double*>(V_in), h->S, h->d.vmax, h->stream);
    } else {
      launch_f32_to_f64(static_cast<const float*>(V_in), h->d.Va64, h->S, h->stream);
      launch_maxabs_f64(h->d.Va64, h->S, h->d.vmax, h->stream);
    }
  }
  const int mode = pi_out ? MODE_GREEDY : MODE_MAX;
  sweep(h, p64, mode, V_in, V_out, p64 ? static_cast<const void*>(h->d.R64) : h->d.R32, nullptr,
        pi_out, nullptr, h->d.slots, nullptr, precision == CPMDP_BF16);
  rc = check_device(h);
  if (rc) return rc;
  if (residual_host) {
    std::vector<double> r;
    rc = read_slots(h, 1, r, nullptr);
    if (rc) return rc;
    *residual_host = r[0];
    if (!std::isfinite(r[0])) return fail(h, CPMDP_E_NONFINITE, "non-finite residual");
  }
  return CPMDP_OK;
}

int cpmdp_policy_backup(cpmdp_t* h, const void* V_in, void* V_out, const int32_t* pi,
                        double* residual_host, int precision) {
  int rc = check_common(h, precision);
  if (rc) return rc;
  if (!V_in || !V_out || !pi) return fail(h, CPMDP_E_ARG, "NULL buffer");
  if (V_in == V_out) return fail(h, CPMDP_E_ARG, "V_in and V_out must not alias");
  rc = check_policy(h, pi);
  if (rc) return rc;
  const bool p64 = precision == CPMDP_FP64;
  zero_slots(h, 1);
  sweep(h, p64, MODE_EVAL, V_in, V_out, p64 ? static_cast<const void*>(h->d.R64) : h->d.R32, pi,
        nullptr, nullptr, h->d.slots, nullptr, precision == CPMDP_BF16);
  rc = check_device(h);
  if (rc) return rc;
  if (residual_host) {
    std::vector<double> r;
    rc = read_slots(h, 1, r, nullptr);
    if (rc) return rc;
    *residual_host = r[0];
  }
  return CPMDP_OK;
}

int cpmdp_value_iteration(cpmdp_t* h, double* V, int32_t* pi_out, double eps, int64_t max_iter,
                          int precision, int64_t* sweeps_out, double* residual_out) {
  int rc = check_common(h, precision);
  if (rc) return rc;
  if (!V) return fail(h, CPMDP_E_ARG, "V is NULL");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(h, CPMDP_E_ARG, "eps must be > 0");
  if (max_iter < 1) return fail(h, CPMDP_E_ARG, "max_iter must be >= 1");
  int64_t sweeps = 0;
  bool done = false;
  double last = INFINITY;
  const hipStream_t st = h->stream;
  SweepTrend trend;   // carried across the precision stages
  bool low_done = false;   // the low-precision sweeps reached eps / 2 themselves
  if (precision != CPMDP_FP64) {
    // Low-precision sweeps until their own rounding floor, then FP64.
    const double ulp = std::ldexp(1.0, -24);
    const double vbound = h->rmax / (1.0 - h->gamma);
    const double floor32 = 8.0 * ulp * std::max(1.0, vbound);
    launch_f64_to_f32(V, h->d.Va32, h->S, st);
    float* cur = h->d.Va32;
    float* alt = h->d.Vb32;
    if (precision == CPMDP_BF16) {
      // BF16 sweeps down to about ten times their own rounding noise (the
      // BF16 operands and intermediate leave about 1e-4 of the value scale
      // per sweep), or until they stall, then FP32
      double tol16 = std::max(std::max(eps, floor32), 1e-3 * std::max(1.0, vbound));
      rc = run_sweeps<float>(h, false, MODE_MAX, cur, alt, h->d.R32, nullptr, tol16, INFINITY,
                             max_iter - 1, &sweeps, &done, &last, true, &trend);
      if (rc) return rc;
      // rmax / (1 - gamma) overstates ||V*|| when rewards take both signs:
      // bound it from the iterate, ||V*|| <= ||V|| + r / (1 - gamma), and go
      // on in BF16 to 1e-3 of that bound (still about ten times the noise)
      // while it lies well below the first tolerance
      if (done && std::isfinite(last) && sweeps < max_iter - 1) {
        double vm = 0.0;
        rc = maxabs_f32(h, cur, &vm);
        if (rc) return rc;
        const double tol16b = std::max(std::max(eps, floor32),
                                       1e-3 * std::max(1.0, vm + last / (1.0 - h->gamma)));
        if (tol16b < 0.5 * tol16) {
          tol16 = tol16b;
          rc = run_sweeps<float>(h, false, MODE_MAX, cur, alt, h->d.R32, nullptr, tol16, INFINITY,
                                 max_iter - 1, &sweeps, &done, &last, true, &trend);
          if (rc) return rc;
        }
      }
      done = done && tol16 <= std::max(eps, floor32);
    }
    double tol32 = std::max(0.5 * eps, floor32);
    double cert_target = 0.5 * eps;   // FP32 residual from which the certificate is tried first
    if (!done) {
      rc = run_sweeps<float>(h, false, MODE_MAX, cur, alt, h->d.R32, nullptr, tol32,
                             floor32 * 4, max_iter - 1, &sweeps, &done, &last, false, &trend);
      if (rc) return rc;
      // rmax / (1 - gamma) bounds ||V*|| loosely when rewards take both signs:
      // take the FP32 rounding floor from the iterate instead,
      // ||V*|| <= ||V|| + r / (1 - gamma), and go on in FP32 while that floor
      // lies well below the first one (12 ulp of the bound: FP32 sweeps stall
      // at 2-7 ulp of ||V|| on the GridWorlds measured).  Only on instances
      // large enough for an FP64 sweep to cost about twice an FP32 one (on
      // cache-resident ones the two cost the same and the extra round trip
      // is the larger cost).
      const bool large = static_cast<double>(h->S) * h->A >= 16777216.0;
      if (large && std::isfinite(last) && last > 0.5 * eps && sweeps < max_iter - 1) {
        double vm = 0.0;
        rc = maxabs_f32(h, cur, &vm);
        if (rc) return rc;
        const double bound = std::max(1.0, vm + last / (1.0 - h->gamma));
        const double f2 = 12.0 * ulp * bound;
        // the FP64 residual of an FP32 iterate exceeds its FP32 residual by
        // a few ulp of ||V||: stop FP32 that far below eps
        cert_target = eps - 4.0 * ulp * bound;
        if (f2 < 0.5 * floor32 && last > std::max(cert_target, f2)) {
          tol32 = std::max(cert_target > 0.0 ? cert_target : 0.5 * eps, f2);
          rc = run_sweeps<float>(h, false, MODE_MAX, cur, alt, h->d.R32, nullptr, tol32, f2 * 4,
                                 max_iter - 1, &sweeps, &done, &last, false, &trend);
          if (rc) return rc;
        }
      }
    }
    low_done = done && tol32 <= cert_target;
    launch_f32_to_f64(cur, V, h->S, st);
  }
  double cert = INFINITY;
  if (precision != CPMDP_FP64 && h->path == CPMDP_PATH_DENSE) {
    // Dense FP64 chains run on the vector ALUs, many times slower than the
    // low-precision chain.  Finish instead by refining the evaluation of the
    // greedy policy: FP64 certificate and policy, FP64 residual r of
    // V = R + gamma P_pi V, low-precision correction sweeps
    // e <- r + gamma P_pi e, V += e; repeat until certified.
    int32_t* pol = pi_out ? pi_out : h->d.piA;
    bool have_pol = false;
    std::vector<double> r;
    for (;;) {
      rc = certify(h, V, pol, have_pol ? pol : nullptr, &cert, nullptr);
      if (rc) return rc;
      have_pol = true;
      ++sweeps;
      if (cert <= eps || sweeps >= max_iter) break;
      zero_slots(h, 1);
      sweep(h, true, MODE_RESID, V, nullptr, h->d.R64, pol, nullptr, h->d.r32, h->d.slots,
            nullptr, false);
      rc = check_device(h);
      if (rc) return rc;
      rc = read_slots(h, 1, r, nullptr);
      if (rc) return rc;
      ++sweeps;
      if (!std::isfinite(r[0])) return fail(h, CPMDP_E_NONFINITE, "non-finite residual");
      launch_fill_f32(h->d.E0, h->S, 0.0f, st);
      float* cur = h->d.E0;
      float* alt = h->d.E1;
      const double tol_e = std::max(0.25 * eps, 1e-3 * r[0]);
      // FP32 chains whatever the precision: each round must resolve e to
      // 1e-3 of ||r||, about the relative rounding of a BF16 chain, which
      // would stall there (BF16 pays in the value-iteration sweeps above)
      rc = run_sweeps<float>(h, false, MODE_EVAL, cur, alt, h->d.r32, pol, tol_e, 0.0,
                             max_iter - 1, &sweeps, &done, &last, false);
      if (rc) return rc;
      launch_add_f32_to_f64(V, cur, h->S, st);
    }
  } else {
    // low-precision sweeps that reached eps / 2 usually leave an FP64
    // residual below eps: certify before any FP64 sweep
    bool sweep64 = !low_done;
    for (;;) {
      if (sweep64) {
        double* cur = V;
        double* alt = h->d.Va64;
        rc = run_sweeps<double>(h, true, MODE_MAX, cur, alt, h->d.R64, nullptr, eps, 0.0,
                                max_iter - 1, &sweeps, &done, &last, false, &trend);
        if (rc) return rc;
        if (cur != V) HIP_TRY(h, hipMemcpyAsync(V, cur, h->S * 8, hipMemcpyDeviceToDevice, st));
      }
      sweep64 = true;
      rc = certify(h, V, pi_out, nullptr, &cert, nullptr);
      if (rc) return rc;
      ++sweeps;
      if (cert <= eps || sweeps >= max_iter) break;
    }
  }
  if (sweeps_out) *sweeps_out = sweeps;
  if (residual_out) *residual_out = cert;
  return cert <= eps ? CPMDP_OK : CPMDP_NOT_CONVERGED;
}

int cpmdp_policy_iteration(cpmdp_t* h, double* V, int32_t* pi, double eps, int64_t max_iter,
                           int precision, int64_t* outer_out, int64_t* sweeps_out,
                           double* residual_out) {
  int rc = check_common(h, precision);
  if (rc) return rc;
  if (!V || !pi) return fail(h, CPMDP_E_ARG, "NULL buffer");
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(h, CPMDP_E_ARG, "eps must be > 0");
  if (max_iter < 1) return fail(h, CPMDP_E_ARG, "max_iter must be >= 1");
  rc = check_policy(h, pi);
  if (rc) return rc;
  const hipStream_t st = h->stream;
  int64_t sweeps = 0, outer = 0;
  const double rmax = h->rmax;
  const double eps_floor = 0.5 * eps * (1.0 - h->gamma);
  // the first policy is usually far from optimal: evaluate it loosely (a
  // tenth of the reward scale), later ones to 0.05 of the certificate
  double eps_eval = std::max(eps_floor, 1e-1 * std::max(rmax, 1e-300));
  double cert = INFINITY;
  bool converged = false, unsettled = false;
  int certified = 0;
  const bool low = precision != CPMDP_FP64;
  const double floor32 =
      8.0 * std::ldexp(1.0, -24) * std::max(1.0, rmax / (1.0 - h->gamma));
  while (sweeps < max_iter) {
    ++outer;
    // ---- evaluation of pi
    if (!low) {
      double* cur = V;
      double* alt = h->d.Va64;
      bool done = false;
      double last = 0;
      rc = run_sweeps<double>(h, true, MODE_EVAL, cur, alt, h->d.R64, pi, eps_eval, 0.0,
                              max_iter - 1, &sweeps, &done, &last, false);
      if (rc) return rc;
      if (cur != V) HIP_TRY(h, hipMemcpyAsync(V, cur, h->S * 8, hipMemcpyDeviceToDevice, st));
    } else {
      for (;;) {
        if (sweeps >= max_iter - 1) break;
        // FP64 residual of the evaluation equation: r = R + g P_pi V - V
        zero_slots(h, 1);
        sweep(h, true, MODE_RESID, V, nullptr, h->d.R64, pi, nullptr, h->d.r32, h->d.slots,
              nullptr, false);
        rc = check_device(h);
        if (rc) return rc;
        std::vector<double> r;
        rc = read_slots(h, 1, r, nullptr);
        if (rc) return rc;
        ++sweeps;
        if (!std::isfinite(r[0])) return fail(h, CPMDP_E_NONFINITE, "non-finite residual");
        if (r[0] <= eps_eval) break;
        // correction e <- r + g P_pi e, from e = 0, in the low precision
        launch_fill_f32(h->d.E0, h->S, 0.0f, st);
        float* cur = h->d.E0;
        float* alt = h->d.E1;
        bool done = false;
        double last = 0;
        // the correction e is small, so FP32 resolves it relative to ||r||;
        // it need not go further than a quarter of the evaluation target
        const double tol_e = std::max(1e-3 * r[0], 0.25 * eps_eval);
        rc = run_sweeps<float>(h, false, MODE_EVAL, cur, alt, h->d.r32, pi, tol_e,
                               precision == CPMDP_BF16 ? INFINITY : 0.0, max_iter - 1, &sweeps,
                               &done, &last, precision == CPMDP_BF16);
        if (rc) return rc;
        launch_add_f32_to_f64(V, cur, h->S, st);
      }
    }
    // ---- improvement (FP64), keeping the incumbent on ties
    unsigned changes = 0;
    rc = certify(h, V, pi, pi, &cert, &changes);
    if (rc) return rc;
    ++sweeps;
    // Stop when pi is unchanged and V is certified.  Once V is certified,
    // remaining changes can only swap actions whose Q-values differ by less
    // than the evaluation error (evaluation is iterative); after
    // kCertifiedRounds such rounds the certified V and its greedy policy are
    // returned.
    if (cert <= eps) ++certified;
    if (cert <= eps && (changes == 0 || certified >= kCertifiedRounds)) {
      converged = true;
      unsettled = changes != 0;
      break;
    }
    if (changes == 0) eps_eval = std::max(eps_floor, 0.05 * cert);
    else eps_eval = std::max(eps_floor, std::min(eps_eval, 0.05 * cert));
  }
  if (outer_out) *outer_out = outer;
  if (sweeps_out) *sweeps_out = sweeps;
  if (residual_out) *residual_out = cert;
  if (!converged) return CPMDP_NOT_CONVERGED;
  return unsettled ? CPMDP_POLICY_UNSETTLED : CPMDP_OK;
}

int cpmdp_bound_shift(cpmdp_t* h, double* V, double* lo_out, double* hi_out) {
  int rc = check_common(h, CPMDP_FP64);
  if (rc) return rc;
  if (!V) return fail(h, CPMDP_E_ARG, "V is NULL");
  const hipStream_t st = h->stream;
  zero_slots(h, 1);
  sweep(h, true, MODE_MAX, V, h->d.Va64, h->d.R64, nullptr, nullptr, nullptr, h->d.slots, nullptr,
        false);
  launch_fill_u64(h->d.vmax + 2, 2, 0ull, st);
  launch_shift_bounds(V, h->d.Va64, h->d.tbits, h->S, h->d.vmax + 2, st);
  rc = check_device(h);
  if (rc) return rc;
  unsigned long long keys[2];
  HIP_TRY(h, hipMemcpyAsync(h->host_slots, h->d.vmax + 2, 16, hipMemcpyDeviceToHost, st));
  HIP_TRY(h, hipStreamSynchronize(st));
  keys[0] = h->host_slots[0];
  keys[1] = h->host_slots[1];
  auto undo = [](unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return bits_to_double(b);
  };
  if (keys[0] == 0 && keys[1] == 0) {   // every state terminal: BV is exact
    HIP_TRY(h, hipMemcpyAsync(V, h->d.Va64, h->S * 8, hipMemcpyDeviceToDevice, st));
    if (lo_out) *lo_out = 0.0;
    if (hi_out) *hi_out = 0.0;
    return CPMDP_OK;
  }
  const double rmax = undo(keys[0]), rmin = -undo(keys[1]);
  if (!std::isfinite(rmax) || !std::isfinite(rmin))
    return fail(h, CPMDP_E_NONFINITE, "non-finite residual in bound_shift");
  const double c = h->gamma / (1.0 - h->gamma);
  launch_apply_shift(V, h->d.Va64, h->d.tbits, h->S, 0.5 * c * (rmin + rmax), st);
  rc = check_device(h);
  if (rc) return rc;
  if (lo_out) *lo_out = c * rmin;
  if (hi_out) *hi_out = c * rmax;
  return CPMDP_OK;
}

int cpmdp_time_sweeps(cpmdp_t* h, void* V_a, void* V_b, int32_t n, int precision, int mode,
                      const int32_t* pi, double* mean_ms) {
  int rc = check_common(h, precision);
  if (rc) return rc;
  if (!V_a || !V_b || V_a == V_b || n < 1 || !mean_ms)
    return fail(h, CPMDP_E_ARG, "bad time_sweeps arguments");
  if (mode != 0 && mode != 1) return fail(h, CPMDP_E_ARG, "mode must be 0 (max) or 1 (policy)");
  if (mode == 1) {
    if (!pi) return fail(h, CPMDP_E_ARG, "policy sweeps need pi");
    rc = check_policy(h, pi);
    if (rc) return rc;
  }
  const bool p64 = precision == CPMDP_FP64;
  const hipStream_t st = h->stream;
  std::vector<hipEvent_t> ev(2 * static_cast<size_t>(n));
  for (auto& e : ev) HIP_TRY(h, hipEventCreate(&e));
  zero_slots(h, 1);
  void* cur = V_a;
  void* alt = V_b;
  // the events take the kernels' own start / stop times (first kernel of the
  // sweep to last), as a kernel trace reports them
  for (int i = 0; i < n; ++i) {
    const LaunchTiming tm{ev[2 * i], ev[2 * i + 1]};
    sweep(h, p64, mode == 0 ? MODE_MAX : MODE_EVAL, cur, alt,
          p64 ? static_cast<const void*>(h->d.R64) : h->d.R32, pi, nullptr, nullptr, h->d.slots,
          nullptr, precision == CPMDP_BF16, &tm,
          (h->path == CPMDP_PATH_STENCIL || h->path == CPMDP_PATH_LISTS) ? h->d.parts
                                                                          : nullptr);
    std::swap(cur, alt);
  }
  rc = check_device(h);
  HIP_TRY(h, hipStreamSynchronize(st));
  double tot = 0.0;
  for (int i = 0; i < n && rc == 0; ++i) {
    float ms = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
    tot += ms;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc) return rc;
  *mean_ms = tot / n;
  return CPMDP_OK;
}

void cpmdp_destroy(cpmdp_t* h) {
  if (!h) return;
  if (h->host_slots) (void)hipHostFree(h->host_slots);
  if (h->host_ctr) (void)hipHostFree(h->host_ctr);
  for (auto e : h->chunk_ev)
    if (e) (void)hipEventDestroy(e);
  delete h;
}

const char* cpmdp_last_error(const cpmdp_t* h) {
  if (h) return h->err.c_str();
  return g_last_error.c_str();
}

}  // extern "C"

// The opaque handle behind cpmdp_t (host side only).
#pragma once

#include <string>
#include <vector>

#include "cpmdp_internal.h"

namespace cpm {

// Device arrays carved out of the caller's workspace.
struct DevPtrs {
  double* R64 = nullptr;
  float* R32 = nullptr;
  uint32_t* tbits = nullptr;
  unsigned long long* slots = nullptr;   // per-sweep residuals (FP64 bits)
  unsigned long long* vmax = nullptr;    // ||V||_inf (FP64 bits) for the tie rule
  unsigned int* counters = nullptr;      // [0] policy changes, [4] bad actions
  double* Va64 = nullptr;                // FP64 ping-pong partner of the caller's V
  float* Va32 = nullptr;
  float* Vb32 = nullptr;
  float* E0 = nullptr;                   // refinement correction ping-pong
  float* E1 = nullptr;
  float* r32 = nullptr;                  // refinement right-hand side
  int32_t* piA = nullptr;                // policy scratch
  double* w64 = nullptr;                 // stencil weights [A][2n+1]
  float* w32 = nullptr;
  double* fac64 = nullptr;               // dense factors, packed per term
  float* fac32 = nullptr;
  uint16_t* facbf = nullptr;             // BF16 bit patterns
  double* lam64 = nullptr;
  float* lam32 = nullptr;
  uint8_t* kinds = nullptr;
  int32_t* term_start = nullptr;
  char* W = nullptr;                     // dense-chain intermediates
  double* parts = nullptr;               // stencil: per-block residuals [kSlots][blocks]
  uint16_t* obs = nullptr;               // stencil with obstacles: blocked directions [S]
  int32_t* l_cols = nullptr;             // lists: column ranges [nslices * A + 1]
  int32_t* l_succ = nullptr;             // lists: successors [columns * 64]
  double* l_p64 = nullptr;               // lists: probabilities [columns * 64]
  float* l_p32 = nullptr;
  double* t_core64 = nullptr;            // TT: padded cores of every (action, dim)
  float* t_core32 = nullptr;
  char* t_X0 = nullptr;                  // TT: bond channels [maxb][S], ping-pong
  char* t_X1 = nullptr;
  char* t_Y = nullptr;                   // TT: P_a V per action [A][S]
};

}  // namespace cpm

struct cpmdp {
  int n = 0;
  int64_t S = 0;
  int A = 0;
  double gamma = 0.0;
  std::vector<int64_t> sizes;
  std::vector<int32_t> ranks;
  std::vector<int32_t> term_start;
  std::vector<double> factors, lambdas, rewards;
  double rmax = 0.0;                     // max_s |R(s)| (set at create)
  std::vector<uint8_t> terminal;
  std::vector<uint8_t> obstacle;         // empty: no obstacles
  std::vector<uint8_t> kinds;
  int path = 0;
  std::vector<double> w;                 // stencil weights [A][2n+1]
  std::vector<double> kw64;              // stencil [wdiff | wbase] for kernel args
  std::vector<float> kw32;
  int32_t st_vec = 1;                    // stencil: states per thread (1 or 4)
  int32_t st_axis = 0;                   // stencil: axis-structured weights
  int32_t st_blocks = 1;                 // stencil: persistent grid size
  int32_t st_states_per_block = 256;
  int32_t st_march = 0;                  // stencil: marching form (see stencil.hip)
  int32_t st_march_tiles = 0, st_march_seg = 0, st_march_blocks = 0;
  // Def. 3 lists path: sliced layout built at create (see lists.hip)
  int32_t l_nslices = 0, l_blocks = 0, l_slices_per_block = 0;
  std::vector<int32_t> l_cols, l_succ;
  std::vector<double> l_prob;
  // Tensor-Train path: bonds [A][n+1]; padded cores (see tt.hip) and the
  // offset of each (action, dim) block in them; padded mode sizes per dim
  std::vector<int32_t> t_bonds;
  std::vector<double> t_core;
  std::vector<int64_t> t_off;
  std::vector<int32_t> t_mm;
  int32_t t_maxb = 1;
  bool opt_march = true;                 // CPMDP_OPT_MARCH
  cpm::GridGeom geom{};
  cpm::ChainGeom cg64{}, cg32{};
  bool bound = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  cpm::DevPtrs d;
  unsigned long long* host_slots = nullptr;  // pinned
  unsigned* host_ctr = nullptr;              // pinned
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};  // chunk residuals copied (per slot half)
  std::string err;
};

namespace cpm {
int fail(cpmdp_t* h, int code, const std::string& msg);
void layout(const cpmdp_t* h, DevPtrs* d, char* base, size_t* total);
void sweep(cpmdp_t* h, bool prec64, int mode, const void* V, void* Vout, const void* R,
           const int32_t* pi_in, int32_t* pi_out, float* r_out, unsigned long long* slot,
           unsigned int* ctr, bool bf16, const LaunchTiming* tm = nullptr,
           double* part = nullptr);
// Blocks of one stencil or lists sweep (the per-block residual words it
// needs).
int stencil_grid(const cpmdp_t* h);
}  // namespace cpm

// Per-state work of the shift/identity (stencil) backup, shared by the
// single-instance kernel (stencil.hip) and the batched kernel (batch.hip).
//
// With every rank term of the form I (x) ... (x) shift (x) ... (x) I, the mode
// products of V with the factors reduce to reading V at the state itself or
// at one axis neighbour (clamped at the grid edge: a move off the grid stays
// put).  Terms of one action that read the same neighbour are summed into one
// weight, so an action is a (2n+1)-point stencil
//     (P_a V)(s) = sum_p w[a][p] V(nbr_p(s)),
// points p: 0 = the state, 1 + 2k = +e_k, 2 + 2k = -e_k.
// A neighbour that is an obstacle counts as the state itself (the move is
// blocked, as at the grid edge): per state, bit p - 1 of obs[s] marks point p.
#pragma once

#include "common.cuh"

namespace cpm {

template <typename T, int VEC>
struct VecOf;
template <>
struct VecOf<float, 4> { using type = float4; };
template <>
struct VecOf<double, 4> { using type = double4; };
template <>
struct VecOf<float, 2> { using type = float2; };
template <>
struct VecOf<double, 2> { using type = double2; };
template <int VEC>
struct IntVec;
template <>
struct IntVec<4> { using type = int4; };
template <>
struct IntVec<2> { using type = int2; };

template <typename T>
__device__ __forceinline__ T comp(const typename VecOf<T, 4>::type& v, int q) {
  return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}
template <typename T>
__device__ __forceinline__ T comp(const typename VecOf<T, 2>::type& v, int q) {
  return q == 0 ? v.x : v.y;
}
__device__ __forceinline__ int icomp(const int4& v, int q) {
  return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w));
}
__device__ __forceinline__ int icomp(const int2& v, int q) { return q == 0 ? v.x : v.y; }

template <typename T>
__device__ __forceinline__ T tnanmax(T a, T b) {
  return (a != a || a > b) ? a : b;
}

// Weights of one instance.
//   axis form: action a = 2k + d differs from the shared vector base[] only at
//     the centre and its own axis-k points (axis[3a..3a+2] = differences at
//     centre, +e_k, -e_k): P_a V = base . nb + 3 terms.  Holds for any axis
//     move whose slip does not depend on the action (the slip GridWorld).
//   full form: full[a * P + p].
//   eval: full table in LDS for per-state action selection.
template <typename T>
struct StencilW {
  const T* base;
  const T* axis;
  const T* full;
  const T* eval;
  int A;
  T gamma;
};

template <typename T>
struct StencilIO {
  const T* V;
  T* Vout;
  const T* R;
  const uint32_t* tbits;
  const int32_t* pi_in;
  int32_t* pi_out;
  float* r_out;
  const uint16_t* obs;   // blocked-direction bits per state, or nullptr
};

// Points of a state whose neighbour is an obstacle read the state itself.
template <typename T, int P>
__device__ __forceinline__ void block_points(T (&nb)[P], unsigned m) {
#pragma unroll
  for (int p = 1; p < P; ++p) nb[p] = ((m >> (p - 1)) & 1u) ? nb[0] : nb[p];
}

// One state: Q-values of Eq. 1, max / argmax (tie rule) or the fixed-policy
// value, and the residual term.
template <typename T, int N, int MODE, bool AXIS>
__device__ __forceinline__ void stencil_state(const StencilW<T>& W, const T (&nb)[2 * N + 1],
                                              T rs, bool term, int pold, T tol, T& out,
                                              int& pnew, T& res, unsigned& changed) {
  constexpr int P = 2 * N + 1;
  const T g = term ? T(0) : W.gamma;
  const T c = nb[0];
  if (MODE == MODE_MAX || MODE == MODE_GREEDY) {
    T best = -INFINITY, qold = -INFINITY;
    int bi = 0;
    auto visit = [&](int act, T acc) {
      if (MODE == MODE_MAX) {
        best = fmax(best, acc);   // a NaN in V still shows in the residual via c
      } else {
        const T q = fma(g, acc, rs);
        tie_update(q, act, tol, best, bi);
        if (act == pold) qold = q;
      }
    };
    if (AXIS) {
      T base = T(0);
#pragma unroll
      for (int p = 0; p < P; ++p) base = fma(W.base[p], nb[p], base);
#pragma unroll
      for (int act = 0; act < 2 * N; ++act) {
        const int k = act >> 1;
        const T* w3 = W.axis + 3 * act;
        T acc = fma(w3[0], nb[0], base);
        acc = fma(w3[1], nb[1 + 2 * k], acc);
        acc = fma(w3[2], nb[2 + 2 * k], acc);
        visit(act, acc);
      }
    } else {
      for (int act = 0; act < W.A; ++act) {
        const T* wa = W.full + act * P;
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
    const T* wa = W.eval + pold * P;
    T acc = T(0);
#pragma unroll
    for (int p = 0; p < P; ++p) acc = fma(wa[p], nb[p], acc);
    out = fma(g, acc, rs);
  }
  if (MODE != MODE_RESID) res = tnanmax(res, fabs(out - c));
}

// 4-word load / store marked non-temporal: the reward words and V' of a
// sweep too large for the caches are touched once, and marking them keeps
// the L2 for the V words that neighbouring tiles read again.
template <typename V4, typename T>
__device__ __forceinline__ V4 load4_stream(const T* p) {
  typedef T nv4 __attribute__((ext_vector_type(4)));
  const nv4 v = __builtin_nontemporal_load(reinterpret_cast<const nv4*>(p));
  V4 o;
  o.x = v.x;
  o.y = v.y;
  o.z = v.z;
  o.w = v.w;
  return o;
}
template <typename V4, typename T>
__device__ __forceinline__ void store4_stream(T* p, const V4& o) {
  typedef T nv4 __attribute__((ext_vector_type(4)));
  const nv4 v = {o.x, o.y, o.z, o.w};
  __builtin_nontemporal_store(v, reinterpret_cast<nv4*>(p));
}
template <typename V2, typename T>
__device__ __forceinline__ V2 load2_stream(const T* p) {
  typedef T nv2 __attribute__((ext_vector_type(2)));
  const nv2 v = __builtin_nontemporal_load(reinterpret_cast<const nv2*>(p));
  V2 o;
  o.x = v.x;
  o.y = v.y;
  return o;
}
template <typename V2, typename T>
__device__ __forceinline__ void store2_stream(T* p, const V2& o) {
  typedef T nv2 __attribute__((ext_vector_type(2)));
  const nv2 v = {o.x, o.y};
  __builtin_nontemporal_store(v, reinterpret_cast<nv2*>(p));
}
// VEC values of a state run as one vector (nontemporal when STREAM)
template <typename T, int VEC, bool STREAM>
__device__ __forceinline__ typename VecOf<T, VEC>::type loadv(const T* p) {
  using VV = typename VecOf<T, VEC>::type;
  if constexpr (!STREAM) return *reinterpret_cast<const VV*>(p);
  else if constexpr (VEC == 4) return load4_stream<VV>(p);
  else return load2_stream<VV>(p);
}
template <typename T, int VEC, bool STREAM>
__device__ __forceinline__ void storev(T* p, const T (&v)[VEC]) {
  using VV = typename VecOf<T, VEC>::type;
  VV o;
  if constexpr (VEC == 4) {
    o.x = v[0];
    o.y = v[1];
    o.z = v[2];
    o.w = v[3];
  } else {
    o.x = v[0];
    o.y = v[1];
  }
  if constexpr (!STREAM) *reinterpret_cast<VV*>(p) = o;
  else if constexpr (VEC == 4) store4_stream(p, o);
  else store2_stream(p, o);
}

// States s .. s+3 along the last dimension (size[n-1] % 4 == 0, s % 4 == 0)
// given their values c4 and the vectors of their +-e_k neighbours for
// k < n-1 (clamped): the last-dimension neighbours come from c4 and the two
// adjacent scalars; then per-state work and stores (R loads and V' stores
// non-temporal when STREAM).  In a row padded past g.last the real state
// g.last - 1 takes itself as its +e_last neighbour (the clamp of the grid
// edge), and the padded lanes are computed but left out of the residual and
// the change count (their stored values are never read by a real state).
template <typename T, int N, int MODE, bool AXIS, bool STREAM = false>
__device__ __forceinline__ void stencil_vec4(const GridGeom& g, const StencilIO<T>& io,
                                             const StencilW<T>& W, int s, int il,
                                             const typename VecOf<T, 4>::type& c4,
                                             const typename VecOf<T, 4>::type (&plus4)[N > 1 ? N - 1 : 1],
                                             const typename VecOf<T, 4>::type (&minus4)[N > 1 ? N - 1 : 1],
                                             T tol, T& res, double& res_d, unsigned& changed,
                                             bool live = true) {
  using V4 = typename VecOf<T, 4>::type;
  constexpr int P = 2 * N + 1;
  const T left = io.V[s - ((il > 0) ? 1 : 0)];
  const T right = io.V[s + ((il + 4 < g.last) ? 4 : 3)];
  const V4 r4 = STREAM ? load4_stream<V4>(io.R + s) : *reinterpret_cast<const V4*>(io.R + s);
  const uint32_t tw = io.tbits[s >> 5] >> (s & 31);
  int4 p4 = make_int4(-1, -1, -1, -1);
  if (MODE != MODE_MAX && io.pi_in) p4 = *reinterpret_cast<const int4*>(io.pi_in + s);
  uint2 ob = make_uint2(0u, 0u);   // 4 x 16-bit blocked-direction masks
  if (io.obs) ob = *reinterpret_cast<const uint2*>(io.obs + s);
  T outv[4];
  int pnv[4];
  unsigned ch = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    T nb[P];
    nb[0] = comp<T>(c4, q);
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
      nb[1 + 2 * k] = comp<T>(plus4[k], q);
      nb[2 + 2 * k] = comp<T>(minus4[k], q);
    }
    const bool real = il + q < g.last;
    nb[1 + 2 * (N - 1)] = (il + q + 1 < g.last) ? (q < 3 ? comp<T>(c4, q + 1) : right)
                                                : comp<T>(c4, q);
    nb[2 + 2 * (N - 1)] = q > 0 ? comp<T>(c4, q - 1) : left;
    if (io.obs) block_points<T, P>(nb, ((q < 2 ? ob.x : ob.y) >> (16 * (q & 1))) & 0xFFFFu);
    const int pold = q == 0 ? p4.x : (q == 1 ? p4.y : (q == 2 ? p4.z : p4.w));
    pnv[q] = 0;
    T rq = res;
    unsigned cq = 0;
    stencil_state<T, N, MODE, AXIS>(W, nb, comp<T>(r4, q), (tw >> q) & 1u, pold, tol, outv[q],
                                    pnv[q], rq, cq);
    if (real) {
      res = rq;
      ch += cq;
    }
  }
  if (!live) return;   // a recomputed chunk: its residual terms repeat a live one's
  changed += ch;
  if (MODE == MODE_RESID) {
    float4 r;
    double d[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      d[q] = static_cast<double>(outv[q]) - static_cast<double>(comp<T>(c4, q));
      if (il + q < g.last) res_d = nanmax(res_d, fabs(d[q]));
    }
    r.x = static_cast<float>(d[0]);
    r.y = static_cast<float>(d[1]);
    r.z = static_cast<float>(d[2]);
    r.w = static_cast<float>(d[3]);
    *reinterpret_cast<float4*>(io.r_out + s) = r;
  } else {
    if (io.Vout) {
      V4 o;
      o.x = outv[0];
      o.y = outv[1];
      o.z = outv[2];
      o.w = outv[3];
      if (STREAM) store4_stream(io.Vout + s, o);
      else *reinterpret_cast<V4*>(io.Vout + s) = o;
    }
    if (MODE == MODE_GREEDY && io.pi_out)
      *reinterpret_cast<int4*>(io.pi_out + s) = make_int4(pnv[0], pnv[1], pnv[2], pnv[3]);
  }
}

// The 2-wide form of stencil_vec4: states s and s + 1 (size[n-1] % 2 == 0,
// s % 2 == 0), half the value registers per thread (the FP64 marching
// sweep, whose 4-wide form holds 120 VGPRs).  Same neighbours, padding and
// residual rules as stencil_vec4.
template <typename T, int N, int MODE, bool AXIS, bool STREAM = false>
__device__ __forceinline__ void stencil_vec2(const GridGeom& g, const StencilIO<T>& io,
                                             const StencilW<T>& W, int s, int il,
                                             const typename VecOf<T, 2>::type& c2,
                                             const typename VecOf<T, 2>::type (&plus2)[N > 1 ? N - 1 : 1],
                                             const typename VecOf<T, 2>::type (&minus2)[N > 1 ? N - 1 : 1],
                                             T tol, T& res, double& res_d, unsigned& changed,
                                             bool live = true) {
  using V2 = typename VecOf<T, 2>::type;
  constexpr int P = 2 * N + 1;
  const T left = io.V[s - ((il > 0) ? 1 : 0)];
  const T right = io.V[s + ((il + 2 < g.last) ? 2 : 1)];
  const V2 r2 = loadv<T, 2, STREAM>(io.R + s);
  const uint32_t tw = io.tbits[s >> 5] >> (s & 31);
  int2 p2 = make_int2(-1, -1);
  if (MODE != MODE_MAX && io.pi_in) p2 = *reinterpret_cast<const int2*>(io.pi_in + s);
  uint32_t ob = 0u;   // 2 x 16-bit blocked-direction masks
  if (io.obs) ob = *reinterpret_cast<const uint32_t*>(io.obs + s);
  T outv[2];
  int pnv[2];
  unsigned ch = 0;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    T nb[P];
    nb[0] = comp<T>(c2, q);
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
      nb[1 + 2 * k] = comp<T>(plus2[k], q);
      nb[2 + 2 * k] = comp<T>(minus2[k], q);
    }
    const bool real = il + q < g.last;
    nb[1 + 2 * (N - 1)] = (il + q + 1 < g.last) ? (q < 1 ? comp<T>(c2, q + 1) : right)
                                                : comp<T>(c2, q);
    nb[2 + 2 * (N - 1)] = q > 0 ? comp<T>(c2, q - 1) : left;
    if (io.obs) block_points<T, P>(nb, (ob >> (16 * q)) & 0xFFFFu);
    const int pold = icomp(p2, q);
    pnv[q] = 0;
    T rq = res;
    unsigned cq = 0;
    stencil_state<T, N, MODE, AXIS>(W, nb, comp<T>(r2, q), (tw >> q) & 1u, pold, tol, outv[q],
                                    pnv[q], rq, cq);
    if (real) {
      res = rq;
      ch += cq;
    }
  }
  if (!live) return;
  changed += ch;
  if constexpr (MODE == MODE_RESID) {
    float2 r;
    double d[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      d[q] = static_cast<double>(outv[q]) - static_cast<double>(comp<T>(c2, q));
      if (il + q < g.last) res_d = nanmax(res_d, fabs(d[q]));
    }
    r.x = static_cast<float>(d[0]);
    r.y = static_cast<float>(d[1]);
    *reinterpret_cast<float2*>(io.r_out + s) = r;
  } else {
    if (io.Vout) storev<T, 2, STREAM>(io.Vout + s, outv);
    if (MODE == MODE_GREEDY && io.pi_out)
      *reinterpret_cast<int2*>(io.pi_out + s) = make_int2(pnv[0], pnv[1]);
  }
}

// The VEC states s .. s+VEC-1 (VEC = 2 or 4 needs m_last % VEC == 0 and
// s % VEC == 0):
// loads, per-state work, stores.  Loads use clamped addresses (at the grid
// edge the neighbour is the state itself), so every load is unconditional.
// STREAM: R loads and V' stores non-temporal (VEC = 4).
template <typename T, int N, int MODE, int VEC, bool AXIS, bool STREAM = false>
__device__ __forceinline__ void stencil_chunk(const GridGeom& g, const StencilIO<T>& io,
                                              const StencilW<T>& W, int s, T tol, T& res,
                                              double& res_d, unsigned& changed,
                                              bool live = true) {
  constexpr int P = 2 * N + 1;
  int idx[N];
  uint32_t rem = static_cast<uint32_t>(s);
#pragma unroll
  for (int k = N - 1; k > 0; --k) {
    const uint32_t q = fdiv(rem, g.div[k]);
    idx[k] = static_cast<int>(rem - q * static_cast<uint32_t>(g.size[k]));
    rem = q;
  }
  idx[0] = static_cast<int>(rem);

  if constexpr (VEC == 1) {
    T nb[P];
    const T c = io.V[s];
    nb[0] = c;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int st = g.stride[k];
      nb[1 + 2 * k] = io.V[s + ((idx[k] < g.size[k] - 1) ? st : 0)];
      nb[2 + 2 * k] = io.V[s - ((idx[k] > 0) ? st : 0)];
    }
    if (io.obs) block_points<T, P>(nb, io.obs[s]);
    const bool term = is_terminal(io.tbits, s);
    const int pold = (MODE == MODE_MAX) ? -1 : (io.pi_in ? io.pi_in[s] : -1);
    T out;
    int pnew = 0;
    unsigned ch = 0;
    stencil_state<T, N, MODE, AXIS>(W, nb, io.R[s], term, pold, tol, out, pnew, res, ch);
    if (!live) return;
    changed += ch;
    if (MODE == MODE_RESID) {
      const double d = static_cast<double>(out) - static_cast<double>(c);
      io.r_out[s] = static_cast<float>(d);
      res_d = nanmax(res_d, fabs(d));
    } else {
      if (io.Vout) io.Vout[s] = out;
      if (MODE == MODE_GREEDY && io.pi_out) io.pi_out[s] = pnew;
    }
  } else if constexpr (VEC == 2) {
    using V2 = typename VecOf<T, 2>::type;
    const V2 c2 = *reinterpret_cast<const V2*>(io.V + s);
    V2 plus2[N > 1 ? N - 1 : 1], minus2[N > 1 ? N - 1 : 1];
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
      const int st = g.stride[k];
      plus2[k] = *reinterpret_cast<const V2*>(io.V + s + ((idx[k] < g.size[k] - 1) ? st : 0));
      minus2[k] = *reinterpret_cast<const V2*>(io.V + s - ((idx[k] > 0) ? st : 0));
    }
    stencil_vec2<T, N, MODE, AXIS, STREAM>(g, io, W, s, idx[N - 1], c2, plus2, minus2, tol, res,
                                           res_d, changed, live);
  } else {
    using V4 = typename VecOf<T, 4>::type;
    const V4 c4 = *reinterpret_cast<const V4*>(io.V + s);
    V4 plus4[N > 1 ? N - 1 : 1], minus4[N > 1 ? N - 1 : 1];
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
      const int st = g.stride[k];
      plus4[k] = *reinterpret_cast<const V4*>(io.V + s + ((idx[k] < g.size[k] - 1) ? st : 0));
      minus4[k] = *reinterpret_cast<const V4*>(io.V + s - ((idx[k] > 0) ? st : 0));
    }
    stencil_vec4<T, N, MODE, AXIS, STREAM>(g, io, W, s, idx[N - 1], c4, plus4, minus4, tol, res,
                                           res_d, changed, live);
  }
}

// Marching form: the VEC (4 or 2) states at plane offset p (p % VEC == 0)
// of planes i_0 in [i_begin, i_end) (a plane = the S / m_0 states of one
// i_0), in order, with the previous, current and next plane's values in
// registers so that the dim-0 neighbours are not fetched again; the plane
// after next is prefetched.  Needs n >= 2 and m_last % VEC == 0; p >= S / m_0
// is a no-op.
template <typename T, int N, int MODE, bool AXIS, int VEC = 4>
__device__ __forceinline__ void march_column(const GridGeom& g, const StencilIO<T>& io,
                                             const StencilW<T>& W, int p, int i_begin, int i_end,
                                             T tol, T& res, double& res_d, unsigned& changed) {
  using VV = typename VecOf<T, VEC>::type;
  const int PL = g.stride[0], m0 = g.size[0];
  if (p >= PL || i_begin >= i_end) return;
  int idx[N];
  uint32_t rem = static_cast<uint32_t>(p);
#pragma unroll
  for (int k = N - 1; k > 0; --k) {
    const uint32_t q = fdiv(rem, g.div[k]);
    idx[k] = static_cast<int>(rem - q * static_cast<uint32_t>(g.size[k]));
    rem = q;
  }
  idx[0] = 0;
  const T* Vp = io.V + p;
  VV prev = *reinterpret_cast<const VV*>(Vp + max(i_begin - 1, 0) * PL);
  VV cur = *reinterpret_cast<const VV*>(Vp + i_begin * PL);
  VV nxt = *reinterpret_cast<const VV*>(Vp + min(i_begin + 1, m0 - 1) * PL);
  for (int i0 = i_begin; i0 < i_end; ++i0) {
    const VV nn = *reinterpret_cast<const VV*>(Vp + min(i0 + 2, m0 - 1) * PL);   // prefetch
    const int s = i0 * PL + p;
    VV plusv[N - 1], minusv[N - 1];
    plusv[0] = nxt;
    minusv[0] = prev;
#pragma unroll
    for (int k = 1; k < N - 1; ++k) {
      const int st = g.stride[k];
      plusv[k] = *reinterpret_cast<const VV*>(io.V + s + ((idx[k] < g.size[k] - 1) ? st : 0));
      minusv[k] = *reinterpret_cast<const VV*>(io.V + s - ((idx[k] > 0) ? st : 0));
    }
    if constexpr (VEC == 4)
      stencil_vec4<T, N, MODE, AXIS, true>(g, io, W, s, idx[N - 1], cur, plusv, minusv, tol, res,
                                           res_d, changed);
    else
      stencil_vec2<T, N, MODE, AXIS, true>(g, io, W, s, idx[N - 1], cur, plusv, minusv, tol, res,
                                           res_d, changed);
    prev = cur;
    cur = nxt;
    nxt = nn;
  }
}

}  // namespace cpm

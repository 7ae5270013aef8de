// NED spreading (eq. (10), first step of the NEDNER pipeline) and its transpose.
//
// Forward: U[q1][q2][n] = sum_m s_m g[m][n] phi(q1 - u_m1) phi(q2 - u_m2) over the W
// nearest grid points per axis (periodic), s_m = h_m/(d1 d2).
//
// Layout of the work: one wavefront owns one column q2 of the oversampled grid,
// one segment of S rows along q1 and 64*TT time samples (TT per lane, time is
// the fastest axis of both g and U, so every load and store is coalesced). It
// sweeps the sensor cells along q1 in order; a sensor in cell row c touches rows
// c-W/2+1 .. c+W/2, so the wave keeps a ring of W rows of accumulators in
// registers and retires row c-W/2+1 as soon as cell row c is done. Unrolling
// the sweep by W makes every ring index a compile-time constant. The sensors a
// wave visits, in sweep order, come from a per-(column, segment) list built at
// plan time, each entry carrying the sensor index and its weight for this
// column. There are no atomics: every output element is written once, by one
// lane, in a fixed order, so the result is bitwise deterministic.
#include "kparams.hpp"

namespace nedner {

template <typename T, int N>
struct VecT;
template <typename T>
struct VecT<T, 1> { typedef T type; };
template <>
struct VecT<float, 2> { typedef float __attribute__((ext_vector_type(2))) type; };
template <>
struct VecT<float, 4> { typedef float __attribute__((ext_vector_type(4))) type; };
template <>
struct VecT<double, 2> { typedef double __attribute__((ext_vector_type(2))) type; };
template <>
struct VecT<double, 4> { typedef double __attribute__((ext_vector_type(4))) type; };

// Load TT consecutive values from p; `valid` of them exist (<= 0: none).
template <int TT, typename R>
__device__ __forceinline__ void load_tt(R (&v)[TT], const R* __restrict__ p, int valid, bool vec) {
  if (vec && valid >= TT) {
    typedef typename VecT<R, TT>::type V;
    V x = *reinterpret_cast<const V*>(p);
    if constexpr (TT == 1) {
      v[0] = x;
    } else {
#pragma unroll
      for (int t = 0; t < TT; ++t) v[t] = x[t];
    }
  } else {
#pragma unroll
    for (int t = 0; t < TT; ++t) v[t] = (t < valid) ? p[t] : R(0);
  }
}

template <int TT, typename R>
__device__ __forceinline__ void store_tt(R* __restrict__ p, const R (&v)[TT], int valid, bool vec) {
  if (vec && valid >= TT) {
    typedef typename VecT<R, TT>::type V;
    V x;
    if constexpr (TT == 1) {
      x = v[0];
    } else {
#pragma unroll
      for (int t = 0; t < TT; ++t) x[t] = v[t];
    }
    *reinterpret_cast<V*>(p) = x;
  } else {
#pragma unroll
    for (int t = 0; t < TT; ++t)
      if (t < valid) p[t] = v[t];
  }
}

__device__ __forceinline__ int floor_div(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

__device__ __forceinline__ int pmod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

template <int W, int TT, typename R, typename WT, typename A>
__global__ __launch_bounds__(256) void k_spread(KP p, const R* __restrict__ g, R* __restrict__ U,
                                                int vec) {
  const int lane = threadIdx.x & 63;
  const int q2 = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (q2 >= p.n2) return;
  const int seg = blockIdx.y;
  const int chunk = blockIdx.z;
  const int S0 = seg * p.S;
  const int S1 = min(S0 + p.S, p.n1);
  const int Vstart = S0 - W / 2;
  const int Vend = S1 + W / 2 - 2;
  const int* __restrict__ cb = p.cellbeg + (size_t)(q2 * p.nseg + seg) * p.CB;
  const int* __restrict__ em = p.ent_m;
  const WT* __restrict__ ew = static_cast<const WT*>(p.ent_w2);
  const WT* __restrict__ w1t = static_cast<const WT*>(p.w1);
  const int Nt = p.Nt;
  const int tb = chunk * 64 * TT + lane * TT;
  const int valid = Nt - tb;
  const bool vv = vec != 0;

  A acc[W][TT];
#pragma unroll
  for (int k = 0; k < W; ++k)
#pragma unroll
    for (int t = 0; t < TT; ++t) acc[k][t] = A(0);

  int e = cb[0];
  const int eall = cb[Vend - Vstart + 1];
  // software pipeline: the next entry's data is in flight while this one is used
  R ng[TT];
  WT nw2 = WT(0);
  int nm = 0;
  if (e < eall) {
    nm = em[e];
    nw2 = ew[e];
    load_tt<TT>(ng, g + (size_t)nm * Nt + tb, valid, vv);
  }
  for (int c0 = floor_div(Vstart, W) * W; c0 <= Vend; c0 += W) {
#pragma unroll
    for (int r = 0; r < W; ++r) {
      const int V = c0 + r;
      if (V < Vstart || V > Vend) continue;
      const int stop = cb[V - Vstart + 1];
      while (e < stop) {
        R cg[TT];
#pragma unroll
        for (int t = 0; t < TT; ++t) cg[t] = ng[t];
        const int cm = nm;
        const WT cw2 = nw2;
        ++e;
        if (e < eall) {
          nm = em[e];
          nw2 = ew[e];
          load_tt<TT>(ng, g + (size_t)nm * Nt + tb, valid, vv);
        }
        const WT* __restrict__ w1 = w1t + (size_t)cm * W;
        A gw[TT];
#pragma unroll
        for (int t = 0; t < TT; ++t) gw[t] = A(cg[t]) * A(cw2);
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const A wk = A(w1[k]);
#pragma unroll
          for (int t = 0; t < TT; ++t) acc[(r + k + W / 2 + 1) % W][t] += wk * gw[t];
        }
      }
      // cell row V is done: virtual row V - W/2 + 1 is complete
      const int slot = (r + W / 2 + 1) % W;
      const int Q = V - W / 2 + 1;
      if (Q >= S0 && Q < S1) {
        R o[TT];
#pragma unroll
        for (int t = 0; t < TT; ++t) o[t] = R(acc[slot][t]);
        store_tt<TT>(U + ((size_t)Q * p.n2 + q2) * Nt + tb, o, valid, vv);
      }
#pragma unroll
      for (int t = 0; t < TT; ++t) acc[slot][t] = A(0);
    }
  }
}

// Transpose of the spreading: g'[m][n] = sum_taps s_m phi(q1-u1) phi(q2-u2) U'[q1][q2][n].
// One wavefront per sensor and time chunk; the W x W taps are read straight
// from the grid (coalesced along time) and summed in a fixed order.
template <int W, int TT, typename R, typename WT, typename A>
__global__ __launch_bounds__(256) void k_gather(KP p, const R* __restrict__ U, R* __restrict__ g,
                                                int vec) {
  const int lane = threadIdx.x & 63;
  const int m = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (m >= p.M) return;
  const int chunk = blockIdx.y;
  const int Nt = p.Nt;
  const int tb = chunk * 64 * TT + lane * TT;
  const int valid = Nt - tb;
  const bool vv = vec != 0;
  const int c1 = p.cell[2 * m];
  const int c2 = p.cell[2 * m + 1];
  const WT* __restrict__ w1 = static_cast<const WT*>(p.w1) + (size_t)m * W;
  const WT* __restrict__ w2 = static_cast<const WT*>(p.w2) + (size_t)m * W;
  A acc[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) acc[t] = A(0);
  for (int k1 = 0; k1 < W; ++k1) {
    const int row = pmod(c1 + k1 - W / 2 + 1, p.n1);
    A ra[TT];
#pragma unroll
    for (int t = 0; t < TT; ++t) ra[t] = A(0);
#pragma unroll
    for (int k2 = 0; k2 < W; ++k2) {
      const int col = pmod(c2 + k2 - W / 2 + 1, p.n2);
      R u[TT];
      load_tt<TT>(u, U + ((size_t)row * p.n2 + col) * Nt + tb, valid, vv);
      const A wk = A(w2[k2]);
#pragma unroll
      for (int t = 0; t < TT; ++t) ra[t] += wk * A(u[t]);
    }
    const A wk = A(w1[k1]);
#pragma unroll
    for (int t = 0; t < TT; ++t) acc[t] += wk * ra[t];
  }
  R o[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) o[t] = R(acc[t]);
  store_tt<TT>(g + (size_t)m * Nt + tb, o, valid, vv);
}

// ---------------------------------------------------------------------------
// dispatch over (precision, W, TT)

template <typename R, typename WT, typename A, int W, int TT>
static hipError_t spread_wt(const KP& p, const void* g, void* U, int vec, hipStream_t s) {
  dim3 grid((p.n2 + 3) / 4, p.nseg, p.nchunk);
  hipLaunchKernelGGL((k_spread<W, TT, R, WT, A>), grid, dim3(256), 0, s,
                     p, static_cast<const R*>(g), static_cast<R*>(U), vec);
  return hipGetLastError();
}

template <typename R, typename WT, typename A, int W, int TT>
static hipError_t gather_wt(const KP& p, const void* U, void* g, int vec, hipStream_t s) {
  dim3 grid((p.M + 3) / 4, p.nchunk);
  hipLaunchKernelGGL((k_gather<W, TT, R, WT, A>), grid, dim3(256), 0, s,
                     p, static_cast<const R*>(U), static_cast<R*>(g), vec);
  return hipGetLastError();
}

template <typename R, typename WT, typename A, int W>
static hipError_t spread_w(const KP& p, const void* g, void* U, int vec, hipStream_t s, bool adj) {
  switch (p.TT) {
    case 1: return adj ? gather_wt<R, WT, A, W, 1>(p, g, U, vec, s) : spread_wt<R, WT, A, W, 1>(p, g, U, vec, s);
    case 2: return adj ? gather_wt<R, WT, A, W, 2>(p, g, U, vec, s) : spread_wt<R, WT, A, W, 2>(p, g, U, vec, s);
    case 4: return adj ? gather_wt<R, WT, A, W, 4>(p, g, U, vec, s) : spread_wt<R, WT, A, W, 4>(p, g, U, vec, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename R, typename WT, typename A>
static hipError_t spread_p(const KP& p, const void* a, void* b, int vec, hipStream_t s, bool adj) {
  switch (p.W) {
    case 2: return spread_w<R, WT, A, 2>(p, a, b, vec, s, adj);
    case 4: return spread_w<R, WT, A, 4>(p, a, b, vec, s, adj);
    case 6: return spread_w<R, WT, A, 6>(p, a, b, vec, s, adj);
    case 8: return spread_w<R, WT, A, 8>(p, a, b, vec, s, adj);
    case 10: return spread_w<R, WT, A, 10>(p, a, b, vec, s, adj);
    case 12: return spread_w<R, WT, A, 12>(p, a, b, vec, s, adj);
    case 14: return spread_w<R, WT, A, 14>(p, a, b, vec, s, adj);
    case 16: return spread_w<R, WT, A, 16>(p, a, b, vec, s, adj);
    default: return hipErrorInvalidValue;
  }
}

static int vec_ok(const KP& p, const void* a, const void* b, size_t esz) {
  const size_t al = (size_t)p.TT * esz;
  if (p.Nt % p.TT) return 0;
  if (((uintptr_t)a % al) || ((uintptr_t)b % al)) return 0;
  return 1;
}

static hipError_t dispatch(const KP& p, const void* a, void* b, hipStream_t s, bool adj) {
  switch (p.prec) {
    case PREC_FP64: return spread_p<double, double, double>(p, a, b, vec_ok(p, a, b, 8), s, adj);
    case PREC_FP32C: return spread_p<float, double, double>(p, a, b, vec_ok(p, a, b, 4), s, adj);
    default: return spread_p<float, float, float>(p, a, b, vec_ok(p, a, b, 4), s, adj);
  }
}

hipError_t launch_spread(const KP& p, const void* g, void* U, hipStream_t s) {
  return dispatch(p, g, U, s, false);
}

hipError_t launch_gather(const KP& p, const void* U, void* g, hipStream_t s) {
  return dispatch(p, U, g, s, true);
}

}  // namespace nedner

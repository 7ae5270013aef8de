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
//
// Templates only: each precision's kernels are instantiated in a translation
// unit of its own (k_spread_f64.hip, k_spread_f32.hip, k_spread_f32c.hip,
// k_spread_f32w.hip) so that they compile in parallel; k_spread.hip holds the
// host-side dispatch, the batch preparation and the equispaced placement.
#pragma once
#include "batch.hpp"

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

// Samples are staged in batches of BE = 4 entries: while the wave accumulates
// the entries of one batch, whose samples sit in this lane's LDS slots, the
// samples of the next batch are in flight into registers; at the batch
// boundary they go to LDS and the loads of the batch after are issued. A wave
// thus waits on global memory once per batch, for loads issued a whole batch
// earlier. Each lane reads back only what it wrote, so no barrier is needed.
//
// Accumulation: in A (float or double registers), or, with KAHAN, as blocked
// compensated float sums (FABsum: Blanchard, Higham and Mary, SIAM J. Sci.
// Comput. 42 (2020)): every grid value of the ring is an unevaluated pair
// hi + lo of floats. Terms enter lo with one fused multiply-add each, exactly
// as in the plain path; after every FOLD entries of the sweep, lo of every
// value (the terms since the last fold plus the previous compensation) is
// added to hi with Kahan's update t = hi + lo, lo' = lo - (t - hi), hi = t,
// which keeps in lo the part the addition lost. A grid value thus sees the
// rounding of a plain float sum only over blocks of at most FOLD terms, and
// the blocks are summed with compensation; hi + lo is rounded to the data
// type once, when the row retires. A fold costs 3 operations per value, so
// the compensation adds 3/FOLD operations per term, against three per term
// for Kahan's update on every term.
// Table pointers are separate __restrict__ parameters so that the compiler
// knows they are read-only for the whole kernel and fetches the wave-uniform
// ones (list entries, first-axis weights) through the scalar cache.
// READ_AHEAD: read the next entry's samples during the current entry (float
// sums only; the batched launch, whose per-problem fields take more
// registers, stays without it: the four extra registers would cost it a
// wavefront per SIMD).
template <int W, int TT, typename R, typename WT, typename A, bool VEC, bool KAHAN, bool READ_AHEAD = true>
__device__ __forceinline__ void spread_body_staged(const KP& p, int bx, const int* __restrict__ cellbeg,
                                                   const int* __restrict__ em, const WT* __restrict__ ew,
                                                   const WT* __restrict__ w1t, const R* __restrict__ g,
                                                   R* __restrict__ U) {
  constexpr int BE = 4;
  __shared__ R stage[4][BE * 64 * TT];
  const int lane = threadIdx.x & 63;
  R* __restrict__ stg = stage[threadIdx.x >> 6] + lane * TT;
  // XCD-aware order: the hardware deals workgroups round-robin to the 8 XCDs;
  // give each XCD a contiguous run of (segment, time chunk) items, segments
  // of one column group consecutive, so that the lists and weights the time
  // chunks of a segment share, and the sensors neighbouring segments and
  // columns share, stay in its L2
  const int G = p.nsegt * p.nchunk;
  const int per = (G + 7) / 8;
  const int L = (bx & 7) * per + (bx >> 3);
  if (L >= G) return;
  const int chunk = L % p.nchunk;
  const int gs = L / p.nchunk;
  // the segment is wave-uniform: keep its fields (and everything the sweep
  // derives from them: bounds, list offsets) in scalar registers
  const int4 sd = reinterpret_cast<const int4*>(p.segd)[gs];
  const int wave = threadIdx.x >> 6;
  const int q2 = __builtin_amdgcn_readfirstlane(sd.x * 4 + wave);
  if (q2 >= p.n2) return;
  const int S0 = __builtin_amdgcn_readfirstlane(sd.y);
  const int S1 = __builtin_amdgcn_readfirstlane(sd.z);
  const int cboff = __builtin_amdgcn_readfirstlane(sd.w);
  const int Vstart = S0 - W / 2;
  const int Vend = S1 + W / 2 - 2;
  const int* __restrict__ cb = cellbeg + cboff + (size_t)__builtin_amdgcn_readfirstlane(wave) * (S1 - S0 + W);
  const int Nt = p.Nt;
  const int tb = chunk * 64 * TT + lane * TT;
  const bool lane_ok = tb < Nt;
  // unsigned lane offset: a uniform row address plus a 32-bit lane offset
  // lets the loads take their base from scalar registers
  const unsigned toff = lane_ok ? unsigned(tb) : 0u;

  static_assert(!KAHAN || sizeof(A) == 4, "the compensated sums are float");
  // acc: the sums (plain), or the low parts lo (KAHAN); hi: the high parts
  constexpr int KW = KAHAN ? W : 1, KT = KAHAN ? TT : 1;
  constexpr int FOLD = 16;
  int since_fold = 0;
  A acc[W][TT];
  A hi[KW][KT];
#pragma unroll
  for (int k = 0; k < W; ++k)
#pragma unroll
    for (int t = 0; t < TT; ++t) acc[k][t] = A(0);
#pragma unroll
  for (int k = 0; k < KW; ++k)
#pragma unroll
    for (int t = 0; t < KT; ++t) hi[k][t] = A(0);

  int e = cb[0];
  const int eall = cb[Vend - Vstart + 1];
  // samples of entries nb .. nb+BE-1, in flight, and the sensor indices of
  // the batch after them, read a batch ahead; the table of sensor indices is
  // padded past its end, so every index read here is valid
  R nx[BE][TT];
  int mp[BE];
  auto issue = [&](int e0) {
    if (e0 < eall) {
#pragma unroll
      for (int j = 0; j < BE; ++j) {
        const R* __restrict__ row = g + (size_t)mp[j] * Nt;
        load_tt<TT>(nx[j], row + toff, TT, VEC);
      }
    }
#pragma unroll
    for (int j = 0; j < BE; ++j) mp[j] = em[e0 + BE + j];
  };
  int nb = e;
#pragma unroll
  for (int j = 0; j < BE; ++j) mp[j] = em[nb + j];
  issue(nb);
  // scalar pipeline: the first-axis weights of the sensor of the next entry
  // and that entry's second-axis weight are read one entry ahead, the sensor
  // index two entries ahead (the index and weight tables are padded past
  // their end, so every read ahead is valid)
  WT wn[W];
  {
    const int m0 = em[e];
#pragma unroll
    for (int k = 0; k < W; ++k) wn[k] = w1t[(size_t)m0 * W + k];
  }
  WT w2n = ew[e];
  int mn = em[e + 1];
  // float sums: the samples of the next entry are read from the staging
  // buffer during this entry's multiply-adds, so that the wait at the next
  // entry finds them there; the four scaled samples take the registers the
  // read needs first (double sums keep one scaled sample at a time)
  constexpr bool PRE = READ_AHEAD && sizeof(A) == 4;
  auto stage_batch = [&]() {
#pragma unroll
    for (int j = 0; j < BE; ++j)
#pragma unroll
      for (int t = 0; t < TT; ++t) stg[j * 64 * TT + t] = nx[j][t];
    nb += BE;
    issue(nb);
  };
  R gn[TT];
  if constexpr (PRE) {
    if (e < eall) {
      stage_batch();
#pragma unroll
      for (int t = 0; t < TT; ++t) gn[t] = stg[(e - (nb - BE)) * 64 * TT + t];
    }
  }
  for (int c0 = floor_div(Vstart, W) * W; c0 <= Vend; c0 += W) {
#pragma unroll
    for (int r = 0; r < W; ++r) {
      const int V = c0 + r;
      if (V < Vstart || V > Vend) continue;
      const int stop = cb[V - Vstart + 1];
      while (e < stop) {
        R gv[TT];
        if constexpr (PRE) {
#pragma unroll
          for (int t = 0; t < TT; ++t) gv[t] = gn[t];
        } else {
          if (e == nb) stage_batch();
          const int j = e - (nb - BE);
#pragma unroll
          for (int t = 0; t < TT; ++t) gv[t] = stg[j * 64 * TT + t];
        }
        WT wc[W];
#pragma unroll
        for (int k = 0; k < W; ++k) wc[k] = wn[k];
        const WT w2c = w2n;
        // wait for this entry's samples and weights here, and keep the next
        // entry's scalar loads behind that wait: a scalar load issued before it
        // would be waited for as well (lgkmcnt(0); vmcnt and expcnt untouched)
        __builtin_amdgcn_s_waitcnt(0xC07F);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < W; ++k) wn[k] = w1t[(size_t)mn * W + k];
        w2n = ew[e + 1];
        mn = em[e + 2];
        if constexpr (PRE) {
          A gt[TT];
#pragma unroll
          for (int t = 0; t < TT; ++t) gt[t] = A(gv[t]) * A(w2c);
          // the next entry's samples (its batch staged first when it starts
          // one; a read past the segment's last entry stays in the buffer)
          if (e + 1 == nb) stage_batch();
#pragma unroll
          for (int t = 0; t < TT; ++t) gn[t] = stg[(e + 1 - (nb - BE)) * 64 * TT + t];
#pragma unroll
          for (int t = 0; t < TT; ++t)
#pragma unroll
            for (int k = 0; k < W; ++k) {
              const int sl = (r + k + W / 2 + 1) % W;
              acc[sl][t] += A(wc[k]) * gt[t];
            }
        } else {
          // one time sample at a time: two registers for the scaled sample
          // instead of 2 TT keep the kernel within four wavefronts per SIMD
#pragma unroll
          for (int t = 0; t < TT; ++t) {
            const A gt = A(gv[t]) * A(w2c);
#pragma unroll
            for (int k = 0; k < W; ++k) {
              const int sl = (r + k + W / 2 + 1) % W;
              acc[sl][t] += A(wc[k]) * gt;
            }
          }
        }
        ++e;
        if constexpr (KAHAN) {
          if (++since_fold == FOLD) {
            since_fold = 0;
#pragma unroll
            for (int sl = 0; sl < W; ++sl)
#pragma unroll
              for (int t = 0; t < TT; ++t) {
                const A tsum = hi[sl][t] + acc[sl][t];
                acc[sl][t] = acc[sl][t] - (tsum - hi[sl][t]);
                hi[sl][t] = tsum;
              }
          }
        }
      }
      const int slot = (r + W / 2 + 1) % W;
      const int Q = V - W / 2 + 1;
      if (Q >= S0 && Q < S1 && lane_ok) {
        R o[TT];
#pragma unroll
        for (int t = 0; t < TT; ++t) o[t] = KAHAN ? R(hi[slot % KW][t % KT] + acc[slot][t]) : R(acc[slot][t]);
        store_tt<TT>(U + ((size_t)Q * p.n2 + q2) * Nt + tb, o, TT, VEC);
      }
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        acc[slot][t] = A(0);
        if constexpr (KAHAN) hi[slot % KW][t % KT] = A(0);
      }
    }
  }
}

template <int W, int TT, typename R, typename WT, typename A, bool VEC, bool KAHAN>
__global__ __launch_bounds__(256) void k_spread(KP p, const int* __restrict__ cellbeg,
                                                const int* __restrict__ em,
                                                const WT* __restrict__ ew,
                                                const WT* __restrict__ w1t,
                                                const R* __restrict__ g, R* __restrict__ U) {
  spread_body_staged<W, TT, R, WT, A, VEC, KAHAN>(p, blockIdx.x, cellbeg, em, ew, w1t, g, U);
}

// Transpose of the spreading: g'[m][n] = sum_taps s_m phi(q1-u1) phi(q2-u2) U'[q1][q2][n].
// A workgroup's four wavefronts handle four consecutive sensors and one time
// chunk (64 TT samples, coalesced along time); each sums its W x W taps in a
// fixed order (along the second axis, then along the first).
//
// Neighbouring sensors read mostly the same grid points. When the four tap
// windows together fit in GC columns and 2W rows, the workgroup stages each
// row of their union in LDS once (the wavefronts loading its columns in turn)
// and every wavefront takes its taps from there, so the grid is read from L2
// about once per workgroup instead of once per sensor. Otherwise each
// wavefront reads its taps directly. Both paths add the same terms in the
// same order: the W taps of a row in the data type R (a fixed W-term dot
// product), the W row sums in the accumulation type A (double for the
// wide-sum FP32 path), with KAHAN in float with Kahan's compensation.
template <int W, int TT, typename R, typename WT, typename A, bool KAHAN>
__device__ __forceinline__ void gather_body(const KP& p, int bx, const R* __restrict__ U,
                                            R* __restrict__ g, int vec) {
  constexpr int GC = W + 12;
  constexpr int SPAN = 64 * TT;
  __shared__ __align__(16) R tile[GC * SPAN];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  // XCD-aware order: each of the 8 XCDs takes a contiguous run of sensor
  // groups of one time chunk, so that neighbouring sensors, which read mostly
  // the same grid rows, share its L2
  const int ngrp = (p.M + 3) / 4;
  const int G = ngrp * p.nchunk;
  const int per = (G + 7) / 8;
  const int L = (bx & 7) * per + (bx >> 3);
  if (L >= G) return;
  const int chunk = L / ngrp;
  // group members: positions m0 .. m0 + 3 of the gather order (tiles of 4 x 4
  // cells), so that they are neighbours whatever the sensors' numbering
  const int m0 = (L - chunk * ngrp) * 4;
  const int* __restrict__ ord = p.gorder;
  const bool act = m0 + wv < p.M;
  const int m = __builtin_amdgcn_readfirstlane(act ? ord[m0 + wv] : 0);
  const int Nt = p.Nt, n1 = p.n1, n2 = p.n2;
  const int tb = chunk * SPAN + lane * TT;
  const int valid = Nt - tb;
  const bool vv = vec != 0;
  const WT* __restrict__ w1 = static_cast<const WT*>(p.w1) + (size_t)m * W;
  const WT* __restrict__ w2 = static_cast<const WT*>(p.w2) + (size_t)m * W;
  // cells of the group's sensors relative to the first one (periodic)
  const int nm = p.M - m0 < 4 ? p.M - m0 : 4;
  const int s0 = ord[m0];
  const int b1 = p.cell[2 * s0], b2 = p.cell[2 * s0 + 1];
  auto rel = [](int d, int n) { return d > n / 2 ? d - n : (d < -n / 2 ? d + n : d); };
  int r_lo = 0, r_hi = 0, c_lo = 0, c_hi = 0, my1 = 0, my2 = 0;
  for (int i = 1; i < nm; ++i) {
    const int si = ord[m0 + i];
    const int d1 = rel(p.cell[2 * si] - b1, n1);
    const int d2 = rel(p.cell[2 * si + 1] - b2, n2);
    r_lo = d1 < r_lo ? d1 : r_lo;
    r_hi = d1 > r_hi ? d1 : r_hi;
    c_lo = d2 < c_lo ? d2 : c_lo;
    c_hi = d2 > c_hi ? d2 : c_hi;
    if (i == wv) {
      my1 = d1;
      my2 = d2;
    }
  }
  const int nr = r_hi - r_lo + W, nc = c_hi - c_lo + W;
  A acc[TT], cmp[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) acc[t] = cmp[t] = A(0);
  // acc += wk ra, compensated with KAHAN
  auto add_row = [&](A wk, const R (&ra)[TT]) {
#pragma unroll
    for (int t = 0; t < TT; ++t) {
      if constexpr (KAHAN) {
        const A y = fmaf(wk, A(ra[t]), -cmp[t]);
        const A s2 = acc[t] + y;
        cmp[t] = (s2 - acc[t]) - y;
        acc[t] = s2;
      } else {
        acc[t] += wk * A(ra[t]);
      }
    }
  };
  if (nc <= GC && nr <= 2 * W) {
    // union row r is grid row b1 + r_lo - W/2 + 1 + r; this sensor's tap k1
    // sits at union row k1 + my1 - r_lo, its tap k2 at union column k2 + my2 - c_lo
    const int base_r = b1 + r_lo - W / 2 + 1, base_c = b2 + c_lo - W / 2 + 1;
    const int k1_0 = my1 - r_lo, k2_0 = my2 - c_lo;
    // this wavefront stages union columns wv, wv + 4, ...; the next row's
    // loads are issued before the current row is summed, so their latency
    // overlaps the sums and the barriers
    constexpr int SL = (GC + 3) / 4;
    R nx[SL][TT];
    auto fetch = [&](int r) {
      const size_t rowoff = (size_t)pmod(base_r + r, n1) * n2;
#pragma unroll
      for (int j = 0; j < SL; ++j) {
        const int sc = wv + 4 * j;
        if (sc < nc) load_tt<TT>(nx[j], U + (rowoff + pmod(base_c + sc, n2)) * Nt + tb, valid, vv);
      }
    };
    fetch(0);
    for (int r = 0; r < nr; ++r) {
#pragma unroll
      for (int j = 0; j < SL; ++j) {
        const int sc = wv + 4 * j;
        if (sc < nc) {
#pragma unroll
          for (int t = 0; t < TT; ++t) tile[sc * SPAN + lane * TT + t] = nx[j][t];
        }
      }
      __syncthreads();
      if (r + 1 < nr) fetch(r + 1);
      const int k1 = r - k1_0;
      if (act && k1 >= 0 && k1 < W) {
        R ra[TT];
#pragma unroll
        for (int t = 0; t < TT; ++t) ra[t] = R(0);
#pragma unroll
        for (int k2 = 0; k2 < W; ++k2) {
          const R* tp = tile + (k2_0 + k2) * SPAN + lane * TT;
          const R wk = R(w2[k2]);
#pragma unroll
          for (int t = 0; t < TT; ++t) ra[t] += wk * tp[t];
        }
        add_row(A(w1[k1]), ra);
      }
      __syncthreads();
    }
  } else {
    if (!act) return;
    const int c1 = p.cell[2 * m];
    const int c2 = p.cell[2 * m + 1];
    for (int k1 = 0; k1 < W; ++k1) {
      const int row = pmod(c1 + k1 - W / 2 + 1, n1);
      R ra[TT];
#pragma unroll
      for (int t = 0; t < TT; ++t) ra[t] = R(0);
#pragma unroll
      for (int k2 = 0; k2 < W; ++k2) {
        const int col = pmod(c2 + k2 - W / 2 + 1, n2);
        R u[TT];
        load_tt<TT>(u, U + ((size_t)row * n2 + col) * Nt + tb, valid, vv);
        const R wk = R(w2[k2]);
#pragma unroll
        for (int t = 0; t < TT; ++t) ra[t] += wk * u[t];
      }
      add_row(A(w1[k1]), ra);
    }
  }
  if (!act) return;
  R o[TT];
#pragma unroll
  for (int t = 0; t < TT; ++t) o[t] = KAHAN ? R(acc[t] - cmp[t]) : R(acc[t]);
  store_tt<TT>(g + (size_t)m * Nt + tb, o, valid, vv);
}

template <int W, int TT, typename R, typename WT, typename A, bool KAHAN>
__global__ __launch_bounds__(256) void k_gather(KP p, const R* __restrict__ U, R* __restrict__ g,
                                                int vec) {
  gather_body<W, TT, R, WT, A, KAHAN>(p, blockIdx.x, U, g, vec);
}

// Transpose of the spreading as a sweep along the first axis, the mirror of
// the forward sweep: a wavefront owns a pair of second-axis cell columns
// (2c, 2c + 1: the sensors whose windows start there read W + 1 grid
// columns), one segment of first-axis cell rows [S0, S1) and 64 time samples
// (one per lane, coalesced). It walks the grid rows in order, keeping the last
// RS rows of its W + 1 columns in registers (a ring, every index compile-time
// by unrolling the walk by RS), and loads each row P = RS - W steps before the
// first sensor that needs it, so the loads of P rows are in flight while the
// sensors of earlier rows are summed. A sensor of cell row V is summed P
// steps after row V + W/2 was loaded: all its W x W taps are then in the ring
// (at column offset 0 or 1 of the pair). Each grid value is loaded once per
// column pair whose windows cover it, from L2 (neighbouring pairs share their
// rows there), and every tap of every sensor is read from registers. The
// terms are added in the order of the tile-staged gather (the W taps of a row
// in R, then the W row sums in A, with KAHAN compensated), so both give the
// same values.
template <int W, int RS, typename R, typename WT, typename A, bool KAHAN>
__global__ __launch_bounds__(256) void k_gather_sweep(KP p, const int* __restrict__ colbeg,
                                                      const int* __restrict__ colm,
                                                      const WT* __restrict__ w1t,
                                                      const WT* __restrict__ w2t,
                                                      const R* __restrict__ U, R* __restrict__ g) {
  constexpr int P = RS - W;
  constexpr int WC = W + 1;  // grid columns of a cell-column pair
  static_assert(P >= 0, "the ring holds at least the W rows of a sensor");
  const int n1 = p.n1, n2 = p.n2, Nt = p.Nt;
  const int npair = (n2 + 1) >> 1;
  const int ngrp = (npair + 3) >> 2;
  const int nsg = (n1 + p.gS - 1) / p.gS;
  const int nch = (Nt + 63) >> 6;
  const int G = ngrp * nsg * nch;
  // XCD-aware order: each XCD takes a contiguous run of items, column groups
  // fastest, so that neighbouring cell columns (which read mostly the same
  // grid columns) sweep the same rows on one XCD at about the same time
  const int per = (G + 7) >> 3;
  const int L = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (L >= G) return;
  const int grp = L % ngrp;
  const int rest = L / ngrp;
  const int sg = rest % nsg;
  const int chunk = rest / nsg;
  const int lane = threadIdx.x & 63;
  const int cp = __builtin_amdgcn_readfirstlane(grp * 4 + (threadIdx.x >> 6));
  if (cp >= npair) return;
  const int S0 = sg * p.gS;
  const int S1 = S0 + p.gS < n1 ? S0 + p.gS : n1;
  const int t = chunk * 64 + lane;
  const bool tok = t < Nt;
  // lanes past the end read sample 0 (a valid address) and store nothing
  const unsigned toff = tok ? unsigned(t) : 0u;
  const int* __restrict__ cb = colbeg + (size_t)cp * (n1 + 1);
  // rows are read with buffer loads: a scalar resource per grid row (its
  // n2 Nt samples), a scalar byte offset per column and one vector byte
  // offset for the lane, so that no load needs a 64-bit vector address
  static_assert(sizeof(R) == 4, "the sweep gather reads 32-bit samples");
  const int rowbytes = n2 * Nt * 4;
  const int voff = int(toff) * 4;
  int soff[WC];
#pragma unroll
  for (int k = 0; k < WC; ++k) soff[k] = pmod(2 * cp - W / 2 + 1 + k, n2) * Nt * 4;
  R ring[RS][WC];
  const int Qa = S0 - W / 2 + 1, Qb = S1 - 1 + W / 2;
  // scalar pipeline: the sensor entry (2 m + column offset) and both weight
  // rows of the next sensor are loaded while the current one is summed, the
  // entry of the one after that a sensor earlier (the sensor table is padded
  // past its end); the list bound of a step's cell row is read a step
  // ahead (the bounds table is padded around every pair's range)
  int e = cb[S0];
  int v_next = colm[e];
  int v_after = colm[e + 1];
  WT w1n[W], w2n[W];
#pragma unroll
  for (int k = 0; k < W; ++k) {
    w1n[k] = w1t[(size_t)(v_next >> 1) * W + k];
    w2n[k] = w2t[(size_t)(v_next >> 1) * W + k];
  }
  // the list bound of the next step's cell row, read a step ahead
  int cb_next = cb[floor_div(Qa, RS) * RS - P - W / 2 + 1];
  for (int q0 = floor_div(Qa, RS) * RS; q0 <= Qb + P; q0 += RS) {
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int q1 = q0 + r;
      const int e_end = cb_next;
      cb_next = cb[q1 - P - W / 2 + 2];
      if (q1 < Qa || q1 > Qb + P) continue;
      // first the sensors whose last row is q1 - P (the newest of their rows
      // was loaded P steps ago), then the loads of row q1 into the slot of
      // row q1 - RS, which no sensor needs any more
      const int V = q1 - P - W / 2;
      if (V >= S0 && V < S1) {
        for (; e < e_end; ++e) {
          // wait for this sensor's scalar loads, and issue the next ones only
          // after the wait (a scalar load issued before it would be waited
          // for as well; lgkmcnt(0), vmcnt and expcnt untouched)
          __builtin_amdgcn_s_waitcnt(0xC07F);
          __builtin_amdgcn_sched_barrier(0);
          const int v = __builtin_amdgcn_readfirstlane(v_next);
          WT w1[W], w2[W];
#pragma unroll
          for (int k = 0; k < W; ++k) {
            w1[k] = w1n[k];
            w2[k] = w2n[k];
          }
          v_next = v_after;
#pragma unroll
          for (int k = 0; k < W; ++k) {
            w1n[k] = w1t[(size_t)(v_next >> 1) * W + k];
            w2n[k] = w2t[(size_t)(v_next >> 1) * W + k];
          }
          v_after = colm[e + 2];
          // the second-axis weights placed at the sensor's column offset in
          // the pair (a zero weight on the other end): one code path for both
          // columns, the extra term adds zero exactly
          const bool odd = (v & 1) != 0;
          WT w2e[WC];
#pragma unroll
          for (int k = 0; k < WC; ++k) {
            const WT lo = k < W ? w2[k] : WT(0);
            const WT hi = k > 0 ? w2[k - 1] : WT(0);
            w2e[k] = odd ? hi : lo;
          }
          A acc = A(0), cmp = A(0);
#pragma unroll
          for (int k1 = 0; k1 < W; ++k1) {
            // row V - W/2 + 1 + k1 = q1 - RS + 1 + k1 sits in slot (r + 1 + k1) mod RS
            const int sl = (r + 1 + k1) % RS;
            R ra = R(0);
#pragma unroll
            for (int k2 = 0; k2 < WC; ++k2) ra += R(w2e[k2]) * ring[sl][k2];
            const A wk = A(w1[k1]);
            if constexpr (KAHAN) {
              const A y = fmaf(wk, A(ra), -cmp);
              const A s2 = acc + y;
              cmp = (s2 - acc) - y;
              acc = s2;
            } else {
              acc += wk * A(ra);
            }
          }
          const R out = KAHAN ? R(acc - cmp) : R(acc);
          if (tok) g[(size_t)(v >> 1) * Nt + t] = out;
        }
      }
      if (q1 <= Qb) {
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<R*>(U + (size_t)pmod(q1, n1) * n2 * Nt), (short)0, rowbytes, 0x00020000);
#pragma unroll
        for (int k = 0; k < WC; ++k)
          ring[r][k] = __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff[k], 0));
      }
    }
  }
}

// ring rows of the sweep gather: W plus rows loaded ahead (0: no sweep for W)
template <int W>
constexpr int sweep_ring() {
  return W <= 12 ? 16 : 0;
}

template <typename R, typename WT, typename A, bool KAHAN, int W>
static hipError_t gather_sweep_w(const KP& p, const void* U, void* g, hipStream_t s) {
  constexpr int RS = sweep_ring<W>();
  if constexpr (RS == 0) {
    return hipErrorInvalidValue;
  } else {
    const long G = (long)(((p.n2 + 1) / 2 + 3) / 4) * ((p.n1 + p.gS - 1) / p.gS) * ((p.Nt + 63) / 64);
    hipLaunchKernelGGL((k_gather_sweep<W, RS, R, WT, A, KAHAN>), dim3(unsigned(8 * ((G + 7) / 8))), dim3(256), 0, s,
                       p, p.gcolbeg, p.gcolm, static_cast<const WT*>(p.w1), static_cast<const WT*>(p.w2),
                       static_cast<const R*>(U), static_cast<R*>(g));
    return hipGetLastError();
  }
}

// ---------------------------------------------------------------------------
// dispatch over (precision, W, TT)

template <typename R, typename WT, typename A, bool KAHAN, int W, int TT>
static hipError_t spread_wt(const KP& p, const void* g, void* U, int vec, hipStream_t s) {
  const int G = p.nsegt * p.nchunk;
  dim3 grid(8 * ((G + 7) / 8));
  const int* cb = p.cellbeg;
  const int* em = p.ent_m;
  const WT* ew = static_cast<const WT*>(p.ent_w2);
  const WT* w1 = static_cast<const WT*>(p.w1);
  if (vec)
    hipLaunchKernelGGL((k_spread<W, TT, R, WT, A, true, KAHAN>), grid, dim3(256), 0, s, p, cb, em, ew, w1,
                       static_cast<const R*>(g), static_cast<R*>(U));
  else
    hipLaunchKernelGGL((k_spread<W, TT, R, WT, A, false, KAHAN>), grid, dim3(256), 0, s, p, cb, em, ew, w1,
                       static_cast<const R*>(g), static_cast<R*>(U));
  return hipGetLastError();
}

template <typename R, typename WT, typename A, bool KAHAN, int W, int TT>
static hipError_t gather_wt(const KP& p, const void* U, void* g, int vec, hipStream_t s) {
  const long G = (long)((p.M + 3) / 4) * p.nchunk;
  dim3 grid(unsigned(8 * ((G + 7) / 8)));
  hipLaunchKernelGGL((k_gather<W, TT, R, WT, A, KAHAN>), grid, dim3(256), 0, s,
                     p, static_cast<const R*>(U), static_cast<R*>(g), vec);
  return hipGetLastError();
}

template <typename R, typename WT, typename A, bool KAHAN, int W>
static hipError_t spread_w(const KP& p, const void* g, void* U, int vec, hipStream_t s, bool adj) {
  switch (p.TT) {
    case 1: return adj ? gather_wt<R, WT, A, KAHAN, W, 1>(p, g, U, vec, s) : spread_wt<R, WT, A, KAHAN, W, 1>(p, g, U, vec, s);
    case 2: return adj ? gather_wt<R, WT, A, KAHAN, W, 2>(p, g, U, vec, s) : spread_wt<R, WT, A, KAHAN, W, 2>(p, g, U, vec, s);
    case 4: return adj ? gather_wt<R, WT, A, KAHAN, W, 4>(p, g, U, vec, s) : spread_wt<R, WT, A, KAHAN, W, 4>(p, g, U, vec, s);
    default: return hipErrorInvalidValue;
  }
}

// The sweep gather where it applies: float data (the ring of double values
// would not fit the registers), tables present, W <= 12.
inline bool use_sweep_gather(const KP& p, size_t rsize) {
  return rsize == 4 && p.gS > 0 && p.gcolbeg && p.gcolm && p.W <= 12;
}

template <typename R, typename WT, typename A, bool KAHAN>
hipError_t spread_p(const KP& p, const void* a, void* b, int vec, hipStream_t s, bool adj) {
  if constexpr (sizeof(R) == 4) {
    if (adj && use_sweep_gather(p, sizeof(R))) {
      switch (p.W) {
        case 2: return gather_sweep_w<R, WT, A, KAHAN, 2>(p, a, b, s);
        case 4: return gather_sweep_w<R, WT, A, KAHAN, 4>(p, a, b, s);
        case 6: return gather_sweep_w<R, WT, A, KAHAN, 6>(p, a, b, s);
        case 8: return gather_sweep_w<R, WT, A, KAHAN, 8>(p, a, b, s);
        case 10: return gather_sweep_w<R, WT, A, KAHAN, 10>(p, a, b, s);
        case 12: return gather_sweep_w<R, WT, A, KAHAN, 12>(p, a, b, s);
        default: return hipErrorInvalidValue;
      }
    }
  }
  switch (p.W) {
    case 2: return spread_w<R, WT, A, KAHAN, 2>(p, a, b, vec, s, adj);
    case 4: return spread_w<R, WT, A, KAHAN, 4>(p, a, b, vec, s, adj);
    case 6: return spread_w<R, WT, A, KAHAN, 6>(p, a, b, vec, s, adj);
    case 8: return spread_w<R, WT, A, KAHAN, 8>(p, a, b, vec, s, adj);
    case 10: return spread_w<R, WT, A, KAHAN, 10>(p, a, b, vec, s, adj);
    case 12: return spread_w<R, WT, A, KAHAN, 12>(p, a, b, vec, s, adj);
    case 14: return spread_w<R, WT, A, KAHAN, 14>(p, a, b, vec, s, adj);
    case 16: return spread_w<R, WT, A, KAHAN, 16>(p, a, b, vec, s, adj);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// batched: one persistent launch over all problems

template <int W, int TT, typename R, typename WT, typename A, bool VEC, bool KAHAN>
__global__ __launch_bounds__(256) void k_spread_many(const BatchProb* __restrict__ bp, WorkList wl) {
  work_loop(wl, [&](int prob, int local) {
    const BatchProb& B = bp[prob];
    const KP& p = B.kp;
    spread_body_staged<W, TT, R, WT, A, VEC, KAHAN, false>(p, local, p.cellbeg, p.ent_m,
                                                    static_cast<const WT*>(p.ent_w2),
                                                    static_cast<const WT*>(p.w1), static_cast<const R*>(B.g),
                                                    static_cast<R*>(B.b0));
  });
}

// resident workgroups of a persistent launch: every CU filled to occupancy
template <typename K>
static int persistent_grid(K kernel, int threads, size_t smem, int total) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(kernel), threads,
                                                  smem) != hipSuccess || per_cu < 1)
    per_cu = 1;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  const long g = (long)per_cu * cus;
  return (int)(g < total ? g : total);
}

template <typename R, typename WT, typename A, bool KAHAN, int W, int TT>
static hipError_t spread_many_wt(const BatchProb* bp, const WorkList& wl, bool vec, hipStream_t s) {
  if (wl.total <= 0) return hipSuccess;
#define NEDNER_SM(V)                                                                            \
  {                                                                                              \
    auto k = k_spread_many<W, TT, R, WT, A, V, KAHAN>;                                           \
    hipLaunchKernelGGL(k, dim3(persistent_grid(k, 256, 0, wl.total)), dim3(256), 0, s, bp, wl);  \
    return hipGetLastError();                                                                    \
  }
  if (vec) NEDNER_SM(true)
  NEDNER_SM(false)
#undef NEDNER_SM
}

template <typename R, typename WT, typename A, bool KAHAN>
hipError_t spread_many_p(const KP& p0, const BatchProb* bp, const WorkList& wl, bool vec,
                                hipStream_t s) {
#define NEDNER_SMW(WV)                                                            \
  case WV:                                                                        \
    switch (p0.TT) {                                                              \
      case 1: return spread_many_wt<R, WT, A, KAHAN, WV, 1>(bp, wl, vec, s);      \
      case 2: return spread_many_wt<R, WT, A, KAHAN, WV, 2>(bp, wl, vec, s);      \
      case 4: return spread_many_wt<R, WT, A, KAHAN, WV, 4>(bp, wl, vec, s);      \
      default: return hipErrorInvalidValue;                                       \
    }
  switch (p0.W) {
    NEDNER_SMW(2)
    NEDNER_SMW(4)
    NEDNER_SMW(6)
    NEDNER_SMW(8)
    NEDNER_SMW(10)
    NEDNER_SMW(12)
    NEDNER_SMW(14)
    NEDNER_SMW(16)
    default: return hipErrorInvalidValue;
  }
#undef NEDNER_SMW
}

// ---------------------------------------------------------------------------
// occupancy of the forward spreading instance a plan launches (aligned data)

template <typename R, typename WT, typename A, bool KAHAN, int W, int TT>
static int occ_wt(const KP& p) {
  (void)p;
  auto k = k_spread<W, TT, R, WT, A, true, KAHAN>;
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, reinterpret_cast<const void*>(k), 256, 0) != hipSuccess)
    return 1;
  return b > 0 ? b : 1;
}

template <typename R, typename WT, typename A, bool KAHAN, int W>
static int occ_w(const KP& p) {
  switch (p.TT) {
    case 1: return occ_wt<R, WT, A, KAHAN, W, 1>(p);
    case 2: return occ_wt<R, WT, A, KAHAN, W, 2>(p);
    case 4: return occ_wt<R, WT, A, KAHAN, W, 4>(p);
    default: return 1;
  }
}

template <typename R, typename WT, typename A, bool KAHAN>
int occ_p(const KP& p) {
  switch (p.W) {
    case 2: return occ_w<R, WT, A, KAHAN, 2>(p);
    case 4: return occ_w<R, WT, A, KAHAN, 4>(p);
    case 6: return occ_w<R, WT, A, KAHAN, 6>(p);
    case 8: return occ_w<R, WT, A, KAHAN, 8>(p);
    case 10: return occ_w<R, WT, A, KAHAN, 10>(p);
    case 12: return occ_w<R, WT, A, KAHAN, 12>(p);
    case 14: return occ_w<R, WT, A, KAHAN, 14>(p);
    case 16: return occ_w<R, WT, A, KAHAN, 16>(p);
    default: return 1;
  }
}

}  // namespace nedner

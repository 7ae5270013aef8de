// Uniform FFT passes around the NER step.
//
// Forward (eq. (10) second half, and the closing inverse FFT of Sec. 3):
//   lat_a : R2C along q2 of the spread grid, keeping k2 = 0..N2/2
//   lat_b : C2C along q1, keeping j1 = -N1/2..N1/2, times the deconvolution
//           1/(phihat1 phihat2) and the time precorrection 1/phihat_t
//   pass_c: inverse C2C along j1 (the two Nyquist representatives are summed)
//   pass_d: C2R along k2 to the real image
// Adjoint: the exact transposes adj_d, adj_c, adj_b, adj_a.
//
// Every pass is a batch of independent lines: a workgroup loads a tile of
// `TB` lines (consecutive along the fastest memory axis, so each row of the
// tile is one contiguous segment) into LDS, transforms along the slow axis
// with the Stockham engine, and writes the tile back with the per-pass
// pre/post-processing fused in. Two real lines are packed into one complex
// line for the real transforms (lat_a, pass_d, adj_d, adj_a).
#include <cstdio>
#include <cstdlib>
#include <algorithm>

#include "batch.hpp"

namespace nedner {

template <typename R>
struct Smem {
  cpx<R>* tw;
  cpx<R>* a;
  cpx<R>* b;  // second buffer of the ping-pong form
};

template <typename R>
__device__ __forceinline__ Smem<R> carve(char* smem, int n, int TB) {
  Smem<R> s;
  s.tw = reinterpret_cast<cpx<R>*>(smem);
  s.a = s.tw + n;
  s.b = s.a + (size_t)n * TB;
  return s;
}

// The batched transform of a pass: ping-pong (one barrier per stage, two
// buffers) or in place (two barriers per stage, one buffer). Returns the
// buffer that holds the result.
template <bool INV, typename R, bool IP>
__device__ __forceinline__ cpx<R>* pass_fft(Smem<R>& sm, const Radices& rd, int TB, int tid, int nth) {
  if constexpr (IP) {
    fft_lds_ip<INV, R, false, 8>(sm.a, rd, TB, TB, 1, sm.tw, tid, nth);
    return sm.a;
  } else {
    return fft_lds<INV, R, false>(sm.a, sm.b, rd, TB, TB, 1, sm.tw, tid, nth);
  }
}

// XCD-aware tile order: the hardware deals workgroups round-robin to the 8
// XCDs, so workgroup b goes to XCD b & 7. Tile L = (b & 7) per + (b >> 3)
// gives each XCD a contiguous run of tiles in (bx fastest, by) order, so that
// the neighbouring tiles along the contiguous axis, which share cache lines
// at their edges, run under the same L2. Returns false past the last tile.
// The first-axis passes (lat_b, adj_b), whose lines are K2 Nt points apart,
// measured faster in launch order (REMAP false) than in contiguous runs.
// PAIR (lateral pass B and its transpose): launch order, except that the
// two tiles of each consecutive pair go to one XCD: their 64-byte rows are
// the two halves of the same cache lines, which one L2 then fetches once,
// while the chip as a whole still streams one region of the array at a time.
// The grid is a multiple of 16 workgroups.
template <bool REMAP = true, bool PAIR = false>
__device__ __forceinline__ bool xcd_tile(int gx, int ntile, int& bx, int& by) {
  const int per = (ntile + 7) >> 3;
  const int b = int(blockIdx.x);
  const int L = REMAP ? (b & 7) * per + (b >> 3)
                      : (PAIR ? (b & ~15) + ((b & 7) << 1) + ((b >> 3) & 1) : b);
  if (L >= ntile) return false;
  by = L / gx;
  bx = L - by * gx;
  return true;
}

// ---------------------------------------------------------------- forward

template <typename R, bool IP>
__device__ __forceinline__ void lat_a_body(const KP& p, int TB, int bx, int by, const R* __restrict__ U,
                                               cpx<R>* __restrict__ V) {
  extern __shared__ __align__(16) char smem[];
  const int n = p.n2, tid = threadIdx.x, nth = blockDim.x;
  Smem<R> sm = carve<R>(smem, n, TB);
  const int q1 = by, pb = bx * TB, npairs = p.Nt / 2;
  load_twiddles(sm.tw, static_cast<const cpx<R>*>(p.tw_n2), n, tid, nth);
  const R* src = U + (size_t)q1 * n * p.Nt;
  const int lsh = __builtin_ctz(TB);
  stage_in<8>(sm.a, n * TB, tid, nth, [&](int i) {
    const int q2 = i >> lsh, pr = pb + (i & (TB - 1));
    cpx<R> z = {R(0), R(0)};
    if (pr < npairs) z = *reinterpret_cast<const cpx<R>*>(src + (size_t)q2 * p.Nt + 2 * pr);
    return z;
  });
  __syncthreads();
  cpx<R>* Z = pass_fft<false, R, IP>(sm, p.r_n2, TB, tid, nth);
  cpx<R>* dst = V + (size_t)q1 * p.K2 * p.Nt;
  for (int i = tid; i < p.K2 * TB; i += nth) {
    const int k = i >> lsh, pp = i & (TB - 1), pr = pb + pp;
    if (pr >= npairs) continue;
    const cpx<R> a = Z[k * TB + pp];
    const cpx<R> b = Z[(k == 0 ? 0 : n - k) * TB + pp];
    const cpx<R> X = {(a.x + b.x) * R(0.5), (a.y - b.y) * R(0.5)};
    const cpx<R> Y = {(a.y + b.y) * R(0.5), (b.x - a.x) * R(0.5)};
    dst[(size_t)k * p.Nt + 2 * pr] = X;
    dst[(size_t)k * p.Nt + 2 * pr + 1] = Y;
  }
}

template <typename R, bool IP>
__global__ __launch_bounds__(512) void k_lat_a(KP p, int TB, int gx, int ntile, const R* __restrict__ U,
                                               cpx<R>* __restrict__ V) {
  int bx, by;
  if (!xcd_tile(gx, ntile, bx, by)) return;
  lat_a_body<R, IP>(p, TB, bx, by, U, V);
}

template <typename R, bool IP>
__device__ __forceinline__ void lat_b_body(const KP& p, int TB, int bx, int by, const cpx<R>* __restrict__ V,
                                               cpx<R>* __restrict__ G) {
  extern __shared__ __align__(16) char smem[];
  const int n = p.n1, tid = threadIdx.x, nth = blockDim.x;
  Smem<R> sm = carve<R>(smem, n, TB);
  const int k2 = by, nb = bx * TB, Nt = p.Nt;
  load_twiddles(sm.tw, static_cast<const cpx<R>*>(p.tw_n1), n, tid, nth);
  const int lsh = __builtin_ctz(TB);
  stage_in<8>(sm.a, n * TB, tid, nth, [&](int i) {
    const int q1 = i >> lsh, nn = nb + (i & (TB - 1));
    cpx<R> z = {R(0), R(0)};
    if (nn < Nt) z = V[((size_t)q1 * p.K2 + k2) * Nt + nn];
    return z;
  });
  __syncthreads();
  cpx<R>* Z = pass_fft<false, R, IP>(sm, p.r_n1, TB, tid, nth);
  const R* d1 = static_cast<const R*>(p.dec1);
  const R* dt = static_cast<const R*>(p.dect);
  const R d2 = static_cast<const R*>(p.dec2)[k2];
  for (int i = tid; i < p.J1 * TB; i += nth) {
    const int je = i >> lsh, t = i & (TB - 1), nn = nb + t;
    if (nn >= Nt) continue;
    const int j1 = je - p.N1 / 2;
    const int k1 = j1 < 0 ? j1 + n : j1;
    G[((size_t)k2 * p.J1 + je) * Nt + nn] = Z[k1 * TB + t] * (d1[je] * d2 * dt[nn]);
  }
}

template <typename R, bool IP>
__global__ __launch_bounds__(512) void k_lat_b(KP p, int TB, int gx, int ntile, const cpx<R>* __restrict__ V,
                                               cpx<R>* __restrict__ G) {
  int bx, by;
  if (!xcd_tile<false, true>(gx, ntile, bx, by)) return;
  lat_b_body<R, IP>(p, TB, bx, by, V, G);
}

template <typename R, bool IP>
__device__ __forceinline__ void pass_c_body(const KP& p, int TB, int bx, int by, const cpx<R>* __restrict__ Z1,
                                                cpx<R>* __restrict__ Z2) {
  extern __shared__ __align__(16) char smem[];
  const int n = p.N1, tid = threadIdx.x, nth = blockDim.x;
  Smem<R> sm = carve<R>(smem, n, TB);
  const int k2 = by, ib = bx * TB, N3 = p.N3;
  load_twiddles(sm.tw, static_cast<const cpx<R>*>(p.tw_N1), n, tid, nth);
  const cpx<R>* src = Z1 + (size_t)k2 * p.J1 * N3;
  const int lsh = __builtin_ctz(TB);
  stage_in<8>(sm.a, n * TB, tid, nth, [&](int i) {
    const int s = i >> lsh, i3 = ib + (i & (TB - 1));
    cpx<R> z = {R(0), R(0)};
    if (i3 < N3) {
      const int j1 = s < n / 2 ? s : s - n;
      z = src[(size_t)(j1 + n / 2) * N3 + i3];
      if (s == n / 2) z = z + src[(size_t)n * N3 + i3];
    }
    return z;
  });
  __syncthreads();
  cpx<R>* Z = pass_fft<true, R, IP>(sm, p.r_N1, TB, tid, nth);
  cpx<R>* dst = Z2 + (size_t)k2 * n * N3;
  for (int i = tid; i < n * TB; i += nth) {
    const int i1 = i >> lsh, t = i & (TB - 1), i3 = ib + t;
    if (i3 < N3) dst[(size_t)i1 * N3 + i3] = Z[i];
  }
}

template <typename R, bool IP>
__global__ __launch_bounds__(512) void k_pass_c(KP p, int TB, int gx, int ntile, const cpx<R>* __restrict__ Z1,
                                                cpx<R>* __restrict__ Z2) {
  int bx, by;
  if (!xcd_tile(gx, ntile, bx, by)) return;
  pass_c_body<R, IP>(p, TB, bx, by, Z1, Z2);
}

template <typename R, bool IP>
__device__ __forceinline__ void pass_d_body(const KP& p, int TB, int bx, int by, const cpx<R>* __restrict__ Z2,
                                                R* __restrict__ vol) {
  extern __shared__ __align__(16) char smem[];
  const int n = p.N2, tid = threadIdx.x, nth = blockDim.x;
  Smem<R> sm = carve<R>(smem, n, TB);
  const int i1 = by, pb = bx * TB, N3 = p.N3, npairs = N3 / 2, h = n / 2;
  load_twiddles(sm.tw, static_cast<const cpx<R>*>(p.tw_N2), n, tid, nth);
  const int lsh = __builtin_ctz(TB);
  // each half-spectrum bin k = 0..n/2 is read once and feeds bins k and
  // n - k (the real bins 0 and n/2 take the two packed depth lines on one bin)
  constexpr int BATCH = 4;
  const int total = (h + 1) * TB;
  for (int base = 0; base < total; base += BATCH * nth) {
    cpx<R> za[BATCH], zb[BATCH];
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int i = base + tid + q * nth;
      const int k = i >> lsh, pr = pb + (i & (TB - 1));
      za[q] = zb[q] = cpx<R>{R(0), R(0)};
      if (i < total && pr < npairs) {
        const size_t o = ((size_t)k * p.N1 + i1) * N3 + 2 * pr;
        za[q] = Z2[o];
        zb[q] = Z2[o + 1];
      }
    }
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int i = base + tid + q * nth;
      if (i >= total) continue;
      const int k = i >> lsh, pp = i & (TB - 1);
      if (k == 0 || k == h) {
        sm.a[k * TB + pp] = cpx<R>{za[q].x, zb[q].x};
      } else {
        sm.a[k * TB + pp] = cpx<R>{za[q].x - zb[q].y, za[q].y + zb[q].x};
        sm.a[(n - k) * TB + pp] = cpx<R>{za[q].x + zb[q].y, zb[q].x - za[q].y};
      }
    }
  }
  __syncthreads();
  cpx<R>* Z = pass_fft<true, R, IP>(sm, p.r_N2, TB, tid, nth);
  R* dst = vol + (size_t)i1 * n * N3;
  for (int i = tid; i < n * TB; i += nth) {
    const int i2 = i >> lsh, pp = i & (TB - 1), pr = pb + pp;
    if (pr < npairs) *reinterpret_cast<cpx<R>*>(dst + (size_t)i2 * N3 + 2 * pr) = Z[i];
  }
}

template <typename R, bool IP>
__global__ __launch_bounds__(512) void k_pass_d(KP p, int TB, int gx, int ntile, const cpx<R>* __restrict__ Z2,
                                                R* __restrict__ vol) {
  int bx, by;
  if (!xcd_tile(gx, ntile, bx, by)) return;
  pass_d_body<R, IP>(p, TB, bx, by, Z2, vol);
}

// ---------------------------------------------------------------- adjoint

template <typename R, bool IP>
__device__ __forceinline__ void adj_d_body(const KP& p, int TB, int bx, int by, const R* __restrict__ vol,
                                               cpx<R>* __restrict__ Z2) {
  extern __shared__ __align__(16) char smem[];
  const int n = p.N2, tid = threadIdx.x, nth = blockDim.x;
  Smem<R> sm = carve<R>(smem, n, TB);
  const int i1 = by, pb = bx * TB, N3 = p.N3, npairs = N3 / 2, h = n / 2;
  load_twiddles(sm.tw, static_cast<const cpx<R>*>(p.tw_N2), n, tid, nth);
  const R* src = vol + (size_t)i1 * n * N3;
  const int lsh = __builtin_ctz(TB);
  stage_in<8>(sm.a, n * TB, tid, nth, [&](int i) {
    const int i2 = i >> lsh, pr = pb + (i & (TB - 1));
    cpx<R> z = {R(0), R(0)};
    if (pr < npairs) z = *reinterpret_cast<const cpx<R>*>(src + (size_t)i2 * N3 + 2 * pr);
    return z;
  });
  __syncthreads();
  cpx<R>* Z = pass_fft<false, R, IP>(sm, p.r_N2, TB, tid, nth);
  for (int i = tid; i < (h + 1) * TB; i += nth) {
    const int k = i >> lsh, pp = i & (TB - 1), pr = pb + pp;
    if (pr >= npairs) continue;
    const cpx<R> a = Z[k * TB + pp];
    const cpx<R> b = Z[(k == 0 ? 0 : n - k) * TB + pp];
    const R al = (k == 0 || k == h) ? R(0.5) : R(1);
    const cpx<R> Va = {(a.x + b.x) * al, (a.y - b.y) * al};
    const cpx<R> Vb = {(a.y + b.y) * al, (b.x - a.x) * al};
    const size_t o = ((size_t)k * p.N1 + i1) * N3 + 2 * pr;
    Z2[o] = Va;
    Z2[o + 1] = Vb;
  }
}

template <typename R, bool IP>
__global__ __launch_bounds__(512) void k_adj_d(KP p, int TB, int gx, int ntile, const R* __restrict__ vol,
                                               cpx<R>* __restrict__ Z2) {
  int bx, by;
  if (!xcd_tile(gx, ntile, bx, by)) return;
  adj_d_body<R, IP>(p, TB, bx, by, vol, Z2);
}

template <typename R, bool IP>
__device__ __forceinline__ void adj_c_body(const KP& p, int TB, int bx, int by, const cpx<R>* __restrict__ Z2,
                                               cpx<R>* __restrict__ Z1) {
  extern __shared__ __align__(16) char smem[];
  const int n = p.N1, tid = threadIdx.x, nth = blockDim.x;
  Smem<R> sm = carve<R>(smem, n, TB);
  const int k2 = by, ib = bx * TB, N3 = p.N3;
  load_twiddles(sm.tw, static_cast<const cpx<R>*>(p.tw_N1), n, tid, nth);
  const cpx<R>* src = Z2 + (size_t)k2 * n * N3;
  const int lsh = __builtin_ctz(TB);
  stage_in<8>(sm.a, n * TB, tid, nth, [&](int i) {
    const int i1 = i >> lsh, i3 = ib + (i & (TB - 1));
    cpx<R> z = {R(0), R(0)};
    if (i3 < N3) z = src[(size_t)i1 * N3 + i3];
    return z;
  });
  __syncthreads();
  cpx<R>* Z = pass_fft<false, R, IP>(sm, p.r_N1, TB, tid, nth);
  cpx<R>* dst = Z1 + (size_t)k2 * p.J1 * N3;
  for (int i = tid; i < p.J1 * TB; i += nth) {
    const int je = i >> lsh, t = i & (TB - 1), i3 = ib + t;
    if (i3 >= N3) continue;
    const int j1 = je - n / 2;
    const int s = j1 < 0 ? j1 + n : j1;
    dst[(size_t)je * N3 + i3] = Z[s * TB + t];
  }
}

template <typename R, bool IP>
__global__ __launch_bounds__(512) void k_adj_c(KP p, int TB, int gx, int ntile, const cpx<R>* __restrict__ Z2,
                                               cpx<R>* __restrict__ Z1) {
  int bx, by;
  if (!xcd_tile(gx, ntile, bx, by)) return;
  adj_c_body<R, IP>(p, TB, bx, by, Z2, Z1);
}

template <typename R, bool IP>
__device__ __forceinline__ void adj_b_body(const KP& p, int TB, int bx, int by, const cpx<R>* __restrict__ G,
                                               cpx<R>* __restrict__ V) {
  extern __shared__ __align__(16) char smem[];
  const int n = p.n1, tid = threadIdx.x, nth = blockDim.x;
  Smem<R> sm = carve<R>(smem, n, TB);
  const int k2 = by, nb = bx * TB, Nt = p.Nt, h1 = p.N1 / 2;
  load_twiddles(sm.tw, static_cast<const cpx<R>*>(p.tw_n1), n, tid, nth);
  const R* d1 = static_cast<const R*>(p.dec1);
  const R* dt = static_cast<const R*>(p.dect);
  const R d2 = static_cast<const R*>(p.dec2)[k2];
  const int lsh = __builtin_ctz(TB);
  stage_in<8>(sm.a, n * TB, tid, nth, [&](int i) {
    const int k1 = i >> lsh, nn = nb + (i & (TB - 1));
    cpx<R> z = {R(0), R(0)};
    if (nn < Nt) {
      // bin k1 holds the kept modes j1 = k1 and j1 = k1 - n that lie in
      // [-N1/2, N1/2]: one of them on the oversampled grid, both of the
      // Nyquist pair at k1 = N1/2 when n = N1 (the equispaced path)
      const R f = d2 * dt[nn];
      if (k1 <= h1) z = G[((size_t)k2 * p.J1 + k1 + h1) * Nt + nn] * (d1[k1 + h1] * f);
      if (k1 - n >= -h1) z = z + G[((size_t)k2 * p.J1 + k1 - n + h1) * Nt + nn] * (d1[k1 - n + h1] * f);
    }
    return z;
  });
  __syncthreads();
  cpx<R>* Z = pass_fft<true, R, IP>(sm, p.r_n1, TB, tid, nth);
  for (int i = tid; i < n * TB; i += nth) {
    const int q1 = i >> lsh, t = i & (TB - 1), nn = nb + t;
    if (nn < Nt) V[((size_t)q1 * p.K2 + k2) * Nt + nn] = Z[i];
  }
}

template <typename R, bool IP>
__global__ __launch_bounds__(512) void k_adj_b(KP p, int TB, int gx, int ntile, const cpx<R>* __restrict__ G,
                                               cpx<R>* __restrict__ V) {
  int bx, by;
  if (!xcd_tile<false, true>(gx, ntile, bx, by)) return;
  adj_b_body<R, IP>(p, TB, bx, by, G, V);
}

template <typename R, bool IP>
__device__ __forceinline__ void adj_a_body(const KP& p, int TB, int bx, int by, const cpx<R>* __restrict__ V,
                                               R* __restrict__ U) {
  extern __shared__ __align__(16) char smem[];
  const int n = p.n2, tid = threadIdx.x, nth = blockDim.x;
  Smem<R> sm = carve<R>(smem, n, TB);
  const int q1 = by, pb = bx * TB, npairs = p.Nt / 2, h2 = p.N2 / 2;
  load_twiddles(sm.tw, static_cast<const cpx<R>*>(p.tw_n2), n, tid, nth);
  const cpx<R>* src = V + (size_t)q1 * p.K2 * p.Nt;
  const int lsh = __builtin_ctz(TB);
  // bins between the two kept halves (oversampled grid) hold no mode
  const int nmid = n - 2 * h2 - 1;
  for (int i = tid; i < nmid * TB; i += nth) sm.a[(h2 + 1) * TB + i] = cpx<R>{R(0), R(0)};
  // each half-spectrum bin k = 0..h2 is read once and feeds bins k and n - k:
  // the real bins (k = 0, and the Nyquist bin n/2 when it is kept, n = N2)
  // take the two half-spectrum terms of the forward on one bin
  constexpr int BATCH = 4;
  const int total = (h2 + 1) * TB;
  for (int base = 0; base < total; base += BATCH * nth) {
    cpx<R> a[BATCH], b[BATCH];
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int i = base + tid + q * nth;
      const int k = i >> lsh, pr = pb + (i & (TB - 1));
      a[q] = b[q] = cpx<R>{R(0), R(0)};
      if (i < total && pr < npairs) {
        a[q] = src[(size_t)k * p.Nt + 2 * pr];
        b[q] = src[(size_t)k * p.Nt + 2 * pr + 1];
      }
    }
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int i = base + tid + q * nth;
      if (i >= total) continue;
      const int k = i >> lsh, pp = i & (TB - 1);
      if (k == 0 || (k == h2 && 2 * h2 == n)) {
        sm.a[k * TB + pp] = cpx<R>{a[q].x, b[q].x};
      } else {
        sm.a[k * TB + pp] = cpx<R>{(a[q].x - b[q].y) * R(0.5), (a[q].y + b[q].x) * R(0.5)};
        sm.a[(n - k) * TB + pp] = cpx<R>{(a[q].x + b[q].y) * R(0.5), (b[q].x - a[q].y) * R(0.5)};
      }
    }
  }
  __syncthreads();
  cpx<R>* Z = pass_fft<true, R, IP>(sm, p.r_n2, TB, tid, nth);
  R* dst = U + (size_t)q1 * n * p.Nt;
  for (int i = tid; i < n * TB; i += nth) {
    const int q2 = i >> lsh, pp = i & (TB - 1), pr = pb + pp;
    if (pr < npairs) *reinterpret_cast<cpx<R>*>(dst + (size_t)q2 * p.Nt + 2 * pr) = Z[i];
  }
}

template <typename R, bool IP>
__global__ __launch_bounds__(512) void k_adj_a(KP p, int TB, int gx, int ntile, const cpx<R>* __restrict__ V,
                                               R* __restrict__ U) {
  int bx, by;
  if (!xcd_tile(gx, ntile, bx, by)) return;
  adj_a_body<R, IP>(p, TB, bx, by, V, U);
}

// ---------------------------------------------------------------- launchers

// Threads of a single-plan pass: in place, a tile of n * TB points needs no
// more than one thread per 8 points, so short transforms run with fewer
// (whole) wavefronts instead of idling half of them in every stage.
static int pass_threads_for(const KP& p, int n, int TB) {
  if (!p.pass_ip) return p.pass_threads;
  const int need = ((n * TB / 8 + 63) / 64) * 64;
  return std::min(p.pass_threads, std::max(64, need));
}

template <typename R>
static size_t smem_for(int n, int TB, bool ip) {
  return (size_t)n * sizeof(cpx<R>) * ((ip ? 1 : 2) * (size_t)TB + 1);
}

#define NEDNER_PASS_LAUNCH(KERNEL, NLEN, GX, GYLINES, IN_T, OUT_T)                                \
  template <typename R>                                                                         \
  static hipError_t run_##KERNEL(const KP& p, const void* in, void* out, hipStream_t s) {        \
    const int n = (NLEN);                                                                       \
    const int TB = pass_lines_for(p, n, (int)sizeof(cpx<R>));                                   \
    const bool ip = p.pass_ip != 0;                                                             \
    const int nth = pass_threads_for(p, n, TB);                                                 \
    const size_t sh = smem_for<R>(n, TB, ip);                                                   \
    const int gx = ((GYLINES) + TB - 1) / TB, ntile = gx * (GX);                                \
    dim3 grid(16 * ((ntile + 15) / 16));                                                        \
    hipError_t e = ip ? allow_smem(KERNEL<R, true>, sh) : allow_smem(KERNEL<R, false>, sh);     \
    if (e != hipSuccess) return e;                                                              \
    if (ip)                                                                                     \
      hipLaunchKernelGGL((KERNEL<R, true>), grid, dim3(nth), sh, s, p, TB, gx, ntile,           \
                         static_cast<const IN_T*>(in), static_cast<OUT_T*>(out));               \
    else                                                                                        \
      hipLaunchKernelGGL((KERNEL<R, false>), grid, dim3(nth), sh, s, p, TB, gx, ntile,          \
                         static_cast<const IN_T*>(in), static_cast<OUT_T*>(out));               \
    return hipGetLastError();                                                                   \
  }

NEDNER_PASS_LAUNCH(k_lat_a, p.n2, p.n1, p.Nt / 2, R, cpx<R>)
NEDNER_PASS_LAUNCH(k_lat_b, p.n1, p.K2, p.Nt, cpx<R>, cpx<R>)
NEDNER_PASS_LAUNCH(k_pass_c, p.N1, p.K2, p.N3, cpx<R>, cpx<R>)
NEDNER_PASS_LAUNCH(k_pass_d, p.N2, p.N1, p.N3 / 2, cpx<R>, R)
NEDNER_PASS_LAUNCH(k_adj_d, p.N2, p.N1, p.N3 / 2, R, cpx<R>)
NEDNER_PASS_LAUNCH(k_adj_c, p.N1, p.K2, p.N3, cpx<R>, cpx<R>)
NEDNER_PASS_LAUNCH(k_adj_b, p.n1, p.K2, p.Nt, cpx<R>, cpx<R>)
NEDNER_PASS_LAUNCH(k_adj_a, p.n2, p.n1, p.Nt / 2, cpx<R>, R)

// ---------------------------------------------------------------- batched
// One persistent kernel for the four forward passes; the stage picks the pass.
// Per problem: transform length n, number of lines, grid height, in and out.
template <typename R, bool IP>
__global__ __launch_bounds__(512) void k_pass_many(const BatchProb* __restrict__ bp, WorkList wl, int stage) {
  work_loop(wl, [&](int prob, int local) {
    const BatchProb& B = bp[prob];
    const KP& p = B.kp;
    const int cs = (int)sizeof(cpx<R>);
    if (stage == ST_LAT_A) {
      const int TB = pass_lines_for(p, p.n2, cs), gx = (p.Nt / 2 + TB - 1) / TB;
      lat_a_body<R, IP>(p, TB, local % gx, local / gx, static_cast<const R*>(B.b0),
                        static_cast<cpx<R>*>(B.b1));
    } else if (stage == ST_LAT_B) {
      const int TB = pass_lines_for(p, p.n1, cs), gx = (p.Nt + TB - 1) / TB;
      lat_b_body<R, IP>(p, TB, local % gx, local / gx, static_cast<const cpx<R>*>(B.b1),
                        static_cast<cpx<R>*>(B.b0));
    } else if (stage == ST_PASS_C) {
      const int TB = pass_lines_for(p, p.N1, cs), gx = (p.N3 + TB - 1) / TB;
      pass_c_body<R, IP>(p, TB, local % gx, local / gx, static_cast<const cpx<R>*>(B.b1),
                         static_cast<cpx<R>*>(B.b0));
    } else {
      const int TB = pass_lines_for(p, p.N2, cs), gx = (p.N3 / 2 + TB - 1) / TB;
      pass_d_body<R, IP>(p, TB, local % gx, local / gx, static_cast<const cpx<R>*>(B.b0),
                         static_cast<R*>(B.out));
    }
  });
}

template <typename R, bool IP>
static hipError_t pass_many_r(const KP& p0, int stage, const BatchProb* bp, const WorkList& wl, size_t smem,
                              hipStream_t s) {
  if (wl.total <= 0) return hipSuccess;
  auto k = k_pass_many<R, IP>;
  hipError_t e = allow_smem(k, smem);
  if (e != hipSuccess) return e;
  int per_cu = 0, dev = 0, cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), p0.pass_threads,
                                                  smem) != hipSuccess || per_cu < 1)
    per_cu = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int grid = (int)std::min<long>((long)per_cu * cus, wl.total);
  hipLaunchKernelGGL(k, dim3(grid), dim3(p0.pass_threads), smem, s, bp, wl, stage);
  return hipGetLastError();
}

hipError_t launch_pass_many(const KP& p0, int stage, const BatchProb* bp, const WorkList& wl, size_t smem,
                            hipStream_t s) {
  if (p0.prec == PREC_FP64)
    return p0.pass_ip ? pass_many_r<double, true>(p0, stage, bp, wl, smem, s)
                      : pass_many_r<double, false>(p0, stage, bp, wl, smem, s);
  return p0.pass_ip ? pass_many_r<float, true>(p0, stage, bp, wl, smem, s)
                    : pass_many_r<float, false>(p0, stage, bp, wl, smem, s);
}

// The two-column lateral grid of the two-dimensional problem (n2 = 2, one kept
// bin k2 = 0): the transform along q2 is the sum of the two columns, and its
// transpose puts the bin's real part on both. One thread per (q1, sample).
template <typename R>
__global__ __launch_bounds__(256) void k_lat_a_two(const R* __restrict__ U, cpx<R>* __restrict__ V, long n1,
                                                   int Nt) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n1 * Nt) return;
  const long q1 = i / Nt, t = i - q1 * Nt;
  V[i] = cpx<R>{U[(2 * q1) * Nt + t] + U[(2 * q1 + 1) * Nt + t], R(0)};
}

template <typename R>
__global__ __launch_bounds__(256) void k_adj_a_two(const cpx<R>* __restrict__ V, R* __restrict__ U, long n1,
                                                   int Nt) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n1 * Nt) return;
  const long q1 = i / Nt, t = i - q1 * Nt;
  const R x = V[i].x;
  U[(2 * q1) * Nt + t] = x;
  U[(2 * q1 + 1) * Nt + t] = x;
}

template <typename R>
static hipError_t run_two(const KP& p, const void* in, void* out, bool adj, hipStream_t s) {
  const long total = (long)p.n1 * p.Nt;
  const dim3 grid(unsigned((total + 255) / 256));
  if (adj)
    hipLaunchKernelGGL(k_adj_a_two<R>, grid, dim3(256), 0, s, static_cast<const cpx<R>*>(in),
                       static_cast<R*>(out), (long)p.n1, p.Nt);
  else
    hipLaunchKernelGGL(k_lat_a_two<R>, grid, dim3(256), 0, s, static_cast<const R*>(in),
                       static_cast<cpx<R>*>(out), (long)p.n1, p.Nt);
  return hipGetLastError();
}

#define NEDNER_PASS_ENTRY(NAME, KERNEL)                                                   \
  hipError_t NAME(const KP& p, const void* in, void* out, hipStream_t s) {                \
    return p.prec == PREC_FP64 ? run_##KERNEL<double>(p, in, out, s)                      \
                               : run_##KERNEL<float>(p, in, out, s);                      \
  }

hipError_t launch_lat_a(const KP& p, const void* in, void* out, hipStream_t s) {
  if (p.n2 == 2 && p.K2 == 1)
    return p.prec == PREC_FP64 ? run_two<double>(p, in, out, false, s) : run_two<float>(p, in, out, false, s);
  return p.prec == PREC_FP64 ? run_k_lat_a<double>(p, in, out, s) : run_k_lat_a<float>(p, in, out, s);
}
NEDNER_PASS_ENTRY(launch_lat_b, k_lat_b)
NEDNER_PASS_ENTRY(launch_pass_c, k_pass_c)
NEDNER_PASS_ENTRY(launch_pass_d, k_pass_d)
NEDNER_PASS_ENTRY(launch_adj_d, k_adj_d)
NEDNER_PASS_ENTRY(launch_adj_c, k_adj_c)
NEDNER_PASS_ENTRY(launch_adj_b, k_adj_b)
hipError_t launch_adj_a(const KP& p, const void* in, void* out, hipStream_t s) {
  if (p.n2 == 2 && p.K2 == 1)
    return p.prec == PREC_FP64 ? run_two<double>(p, in, out, true, s) : run_two<float>(p, in, out, true, s);
  return p.prec == PREC_FP64 ? run_k_adj_a<double>(p, in, out, s) : run_k_adj_a<float>(p, in, out, s);
}

}  // namespace nedner

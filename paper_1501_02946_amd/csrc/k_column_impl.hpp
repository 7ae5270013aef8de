// NER step (eq. (6)-(8)) fused with the inversion weight of eq. (1), one
// workgroup per column (j1, k2) of the NED result.
//
// Forward, per column:
//   a[n'] = G(n' + Nt/2), n' in [-Nt/2, Nt/2), stored at n' mod ntt, zero padded
//           (G already carries 1/phihat_t, applied in the lateral pass);
//   B = FFT_ntt(a) in LDS;
//   for l in -N3/2..N3/2 (both depth Nyquist representatives):
//     x = omega dt ntt/(2 pi) = sign(l) c dt ntt |K|/(2 pi), reduced in double;
//     H = sum over the W grid points q nearest x of B[q mod ntt] phi(x - q);
//     F = scale * W(j,l) * H * exp(-i (Nt/2 theta + omega t0)), phase in double;
//   then either the spectrum is written out, or the Nyquist combination of
//   the half-spectrum inverse (see column_policy) is applied and the inverse
//   FFT along depth is done in LDS, so the column leaves as Z1.
// Adjoint, per column: the exact transpose, with the interpolation turned
// into a deterministic gather over the monotone sequence x(l).
// With p.cosm the same kernels evaluate the forward operator Q of Sec. 2 on
// the periodic voxel grid (adjoint kernel) and its adjoint (forward kernel):
// each Fourier mode of the initial pressure oscillates as cos(c|K|t) =
// (exp(i omega t) + exp(-i omega t))/2, and since x(-l) = -x(l) the second
// exponential is the first one at -l, so the per-l values are averaged
// between l and -l and weighted by a constant instead of W(j,l). The depth
// mode l = 0 oscillates at c|k| (not at the reconstruction's omega = 0), so
// it is evaluated at the two points +-x0 = +-c dt ntt |k|/(2 pi), which lie
// between x(-1) and x(1) and keep the sequence of points monotone.
//
// Templates only: each precision is instantiated in a translation unit of
// its own (k_column_f64.hip, k_column_f32.hip, k_column_f32p.hip) so the
// three compile in parallel; k_column.hip holds the host-side dispatch.
#pragma once
#include <algorithm>

#include "batch.hpp"

namespace nedner {

__device__ __forceinline__ int pmodc(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// How column (je, k2) enters the half-spectrum inverse transform.
//   fac: overall factor; pol: depth Nyquist slot gets F(-N3/2) (0), F(+N3/2) (1)
//   or their mean (2). The real part of the full inverse DFT equals a C2R along
//   the second axis of the symmetrised half spectrum; at the Nyquist indices the
//   symmetrisation averages the two representatives -N/2 and +N/2.
__device__ __forceinline__ void column_policy(int je, int k2, int N1, int N2, double& fac, int& pol) {
  const bool lo = je == 0, hi = je == N1;
  if (k2 == 0) {
    fac = hi ? 0.0 : 1.0;
    pol = 0;
  } else if (k2 == N2 / 2) {
    fac = lo ? 0.0 : 1.0;
    pol = 1;
  } else if (lo) {
    fac = 0.5;
    pol = 0;
  } else if (hi) {
    fac = 0.5;
    pol = 1;
  } else {
    fac = 1.0;
    pol = 2;
  }
}

template <typename R>
__device__ __forceinline__ R wexp(R v);
template <>
__device__ __forceinline__ float wexp<float>(float v) { return __expf(v); }
template <>
__device__ __forceinline__ double wexp<double>(double v) { return exp(v); }

template <typename R>
__device__ __forceinline__ void sincos_pi(R v, R* s, R* c);
template <>
__device__ __forceinline__ void sincos_pi<float>(float v, float* s, float* c) { sincospif(v, s, c); }
template <>
__device__ __forceinline__ void sincos_pi<double>(double v, double* s, double* c) { sincospi(v, s, c); }

// Modified Bessel function I0 for the Kaiser-Bessel window taps.
// float: the polynomial approximations 9.8.1 (|y| <= 3.75) and 9.8.2 (y > 3.75,
// for sqrt(y) exp(-y) I0(y)) of Abramowitz and Stegun, Handbook of Mathematical
// Functions, relative error below 4e-7; double: the power series
// sum_k (y^2/4)^k / (k!)^2, summed until a term no longer changes the sum.
__device__ __forceinline__ float bessel_i0(float y) {
  if (y <= 3.75f) {
    const float t = (y * (1.0f / 3.75f)) * (y * (1.0f / 3.75f));
    return 1.0f + t * (3.5156229f + t * (3.0899424f + t * (1.2067492f + t * (0.2659732f +
           t * (0.0360768f + t * 0.0045813f)))));
  }
  const float u = 3.75f / y;
  const float q = 0.39894228f + u * (0.01328592f + u * (0.00225319f + u * (-0.00157565f + u * (0.00916281f +
                  u * (-0.02057706f + u * (0.02635537f + u * (-0.01647633f + u * 0.00392377f)))))));
  return q * expf(y) * rsqrtf(y);
}

__device__ __forceinline__ double bessel_i0(double y) {
  const double q = 0.25 * y * y;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 1000; ++k) {
    term *= q / (double(k) * double(k));
    const double next = sum + term;
    if (next == sum) break;
    sum = next;
  }
  return sum;
}

// Kaiser-Bessel tap at offset d (grid units): I0(beta sqrt(1 - (2d/W)^2)) for
// |d| < W/2, else 0; twow = 2/W.
template <typename R>
__device__ __forceinline__ R kb_tap(R d, R beta, R twow) {
  const R a = d * twow;
  const R s = R(1) - a * a;
  return s > R(0) ? bessel_i0(beta * sqrt(s)) : R(0);
}

// Frequency data of one output l of a column: grid position x = q0 + fr,
// the weight W(j,l) times the scale, and exp(-i phase).
template <typename R, bool ARGS64>
struct LPoint {
  int q0;
  R fr;
  R wgt;
  cpx<R> ph;
};

template <typename R, bool ARGS64>
__device__ __forceinline__ LPoint<R, ARGS64> lpoint(const KP& p, double a, int l, double scale) {
  LPoint<R, ARGS64> o;
  const double l2 = double(l) * double(l);
  R rr;
  if constexpr (ARGS64 && sizeof(R) == 4) {
    // float data: |K| in double from a float reciprocal square root and one
    // Newton step (relative error ~1e-14, far below what x needs), x and the
    // phase reduced in double; the weight, which only scales a float value,
    // in float; sin and cos of the reduced phase (in turns) by the hardware
    const double s2 = a + l2 * p.bz;
    const float y = s2 > 0.0 ? __builtin_amdgcn_rsqf(float(s2)) : 0.0f;
    double kk = s2 * double(y);
    kk = fma(0.5 * double(y), fma(-kk, kk, s2), kk);
    const double x = (l > 0 ? 1.0 : (l < 0 ? -1.0 : 0.0)) * p.cdtnt * kk;
    const double fl = floor(x);
    o.q0 = int(fl);
    o.fr = R(x - fl);
    double r = x * p.phase_p;
    r -= rint(r);
    const float rf = float(r);
    float w = 0.0f;
    if (l != 0)
      w = float(p.two_c * sqrt(p.bz)) * fabsf(float(l)) * __builtin_amdgcn_rcpf(float(kk));
    else if (a == 0.0)
      w = float(p.two_c);
    o.wgt = R(w * float(scale));
    o.ph = cpx<R>{__builtin_amdgcn_cosf(rf), -__builtin_amdgcn_sinf(rf)};
    return o;
  } else if constexpr (ARGS64) {
    const double kk = sqrt(a + l2 * p.bz);
    const double x = (l > 0 ? 1.0 : (l < 0 ? -1.0 : 0.0)) * p.cdtnt * kk;
    const double fl = floor(x);
    o.q0 = int(fl);
    o.fr = R(x - fl);
    double r = x * p.phase_p;
    r -= rint(r);
    rr = R(r);
    double w = 0.0;
    if (l != 0)
      w = p.two_c * fabs(double(l)) * sqrt(p.bz) / kk;
    else if (a == 0.0)
      w = p.two_c;
    o.wgt = R(w * scale);
  } else {
    const float kk = sqrtf(float(a) + float(l2) * float(p.bz));
    const float x = (l > 0 ? 1.0f : (l < 0 ? -1.0f : 0.0f)) * float(p.cdtnt) * kk;
    const float fl = floorf(x);
    o.q0 = int(fl);
    o.fr = R(x - fl);
    float r = x * float(p.phase_p);
    r -= rintf(r);
    rr = R(r);
    float w = 0.0f;
    if (l != 0)
      w = float(p.two_c) * fabsf(float(l)) * sqrtf(float(p.bz)) / kk;
    else if (a == 0.0)
      w = float(p.two_c);
    o.wgt = R(w * float(scale));
  }
  R s, c;
  sincos_pi<R>(R(2) * rr, &s, &c);
  o.ph = cpx<R>{c, -s};
  return o;
}

// Grid position, phase and zero weight of the time frequency at x (grid units).
template <typename R, bool ARGS64>
__device__ __forceinline__ LPoint<R, ARGS64> lpoint_at(const KP& p, double x) {
  LPoint<R, ARGS64> o;
  R rr;
  if constexpr (ARGS64) {
    const double fl = floor(x);
    o.q0 = int(fl);
    o.fr = R(x - fl);
    double r = x * p.phase_p;
    r -= rint(r);
    rr = R(r);
  } else {
    const float xf = float(x);
    const float fl = floorf(xf);
    o.q0 = int(fl);
    o.fr = R(xf - fl);
    float r = xf * float(p.phase_p);
    r -= rintf(r);
    rr = R(r);
  }
  o.wgt = R(0);
  R s, c;
  sincos_pi<R>(R(2) * rr, &s, &c);
  o.ph = cpx<R>{c, -s};
  return o;
}

// x0 = c dt ntt |k| / (2 pi) of the lateral mode with squared frequency a,
// in the precision lpoint uses for x.
template <bool ARGS64>
__device__ __forceinline__ double x_lateral(const KP& p, double a) {
  if constexpr (ARGS64)
    return p.cdtnt * sqrt(a);
  else
    return double(float(p.cdtnt) * sqrtf(float(a)));
}

// LDS of one workgroup: the twiddle tables, shared, then per column the
// transform buffer and, unless the forward kernel keeps its per-l values in
// registers, the per-l arrays. The tables hold half a period each
// (tw[i + n/2] = -tw[i]); the depth transform reads the time transform's
// table with stride ntt/N3 when N3 divides ntt, else a table of its own.
// Smaller shared tables leave room for more columns per CU.
template <typename R>
struct ColSmem {
  cpx<R>* twt;    // ntt/2 twiddles
  cpx<R>* tw3;    // N3/2 twiddles (= twt when N3 divides ntt)
  cpx<R>* a;      // nbuf: the transform buffer (in place)
  cpx<R>* fl;     // N3 + 2: one value per output l, and the second l = 0 point of Q
  R* fr;          // N3 + 2 (adjoint)
  int* q0;        // N3 + 2 (adjoint)
  short* st;      // ntt + 2 (adjoint): number of points below each grid cell
};

__host__ __device__ inline bool col_tw3_shared(int ntt, int N3) { return ntt % N3 == 0; }

// The forward kernel holds the N3 + 1 values of a column in registers when
// they fit (N3 + 1 <= 64 NL_REG, NL_REG per lane with one wavefront per
// column, fewer with more); the transform buffer then is all the LDS a
// column needs, which doubles the columns resident per CU.
constexpr int NL_REG = 9;
__host__ __device__ inline bool col_fl_in_regs(int N3) { return N3 + 1 <= 64 * NL_REG; }

// Wavefronts per column: one for transforms up to 512 points (a wavefront
// holds them in 8 points per lane), four above, so that a column's stages
// run on 256 threads and a CU holds more wavefronts than it has columns'
// worth of LDS. Shared by the single and the batched launches.
__host__ __device__ inline int column_wpc(int ntt, int N3) { return (ntt > N3 ? ntt : N3) > 512 ? 4 : 1; }

// Points of a column's transform buffer: the longer transform and the tap
// extension.
__host__ __device__ inline int col_nbuf(int ntt, int N3) { return (ntt > N3 ? ntt : N3) + COL_EXT; }

template <typename R>
__host__ __device__ inline size_t col_wave_bytes(int ntt, int N3, bool adj) {
  const size_t nbuf = col_nbuf(ntt, N3);
  size_t b = sizeof(cpx<R>) * nbuf;
  if (adj || !col_fl_in_regs(N3))
    b += (sizeof(cpx<R>) + sizeof(R) + sizeof(int)) * ((size_t)N3 + 2);
  if (adj) b += sizeof(short) * ((size_t)ntt + 2);
  return (b + 15) & ~size_t(15);
}

template <typename R>
__host__ __device__ inline size_t col_shared_bytes(int ntt, int N3) {
  const size_t n = (size_t)ntt / 2 + (col_tw3_shared(ntt, N3) ? 0 : (size_t)N3 / 2);
  return (sizeof(cpx<R>) * n + 15) & ~size_t(15);
}

// The column's two twiddle accessors and the staging of their tables.
template <typename R>
__device__ __forceinline__ void col_twiddles(const ColSmem<R>& sm, const KP& p, int tid, int nth) {
  load_twiddles(sm.twt, static_cast<const cpx<R>*>(p.tw_ntt), p.ntt / 2, tid, nth);
  if (!col_tw3_shared(p.ntt, p.N3)) load_twiddles(sm.tw3, static_cast<const cpx<R>*>(p.tw_N3), p.N3 / 2, tid, nth);
}
template <typename R>
__device__ __forceinline__ TwHalf<R> col_twt(const ColSmem<R>& sm, const KP& p) {
  return TwHalf<R>{sm.twt, 1, p.ntt / 2};
}
template <typename R>
__device__ __forceinline__ TwHalf<R> col_tw3(const ColSmem<R>& sm, const KP& p) {
  return col_tw3_shared(p.ntt, p.N3) ? TwHalf<R>{sm.twt, p.ntt / p.N3, p.ntt / 2} : TwHalf<R>{sm.tw3, 1, p.N3 / 2};
}

template <typename R>
__device__ __forceinline__ ColSmem<R> col_carve(char* smem, const KP& p, int column, bool adj) {
  ColSmem<R> s;
  const int nbuf = col_nbuf(p.ntt, p.N3);
  s.twt = reinterpret_cast<cpx<R>*>(smem);
  s.tw3 = col_tw3_shared(p.ntt, p.N3) ? s.twt : s.twt + p.ntt / 2;
  char* w = smem + col_shared_bytes<R>(p.ntt, p.N3) + (size_t)column * col_wave_bytes<R>(p.ntt, p.N3, adj);
  s.a = reinterpret_cast<cpx<R>*>(w);
  s.fl = s.a + nbuf;
  s.fr = reinterpret_cast<R*>(s.fl + p.N3 + 2);
  s.q0 = reinterpret_cast<int*>(s.fr + p.N3 + 2);
  s.st = reinterpret_cast<short*>(s.q0 + p.N3 + 2);
  return s;
}

// WPC wavefronts per column (CN = 64 WPC threads); a workgroup of CPW columns
// shares the twiddles. With one wavefront per column a column waits only on
// its own LDS traffic; with several, every stage ends at a workgroup barrier,
// which every column of the workgroup reaches: a column past the end of the
// list, or one the half-spectrum inverse leaves out, runs the same steps on
// zeros and writes nothing.
// SPEC: write the full spectrum F (N1, N2, N3) in FFT order instead of Z1.
template <typename R, int W, bool ARGS64, bool SPEC, int PPT, bool KBW, int WPC>
__device__ __forceinline__ void column_body(const KP& p, int ncol, int bx, const cpx<R>* __restrict__ G,
                                            void* out) {
  extern __shared__ __align__(16) char smem[];
  constexpr int CN = 64 * WPC;
  constexpr bool WV = WPC == 1;
  constexpr int NLW = (NL_REG + WPC - 1) / WPC;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int ct = tid % CN, cw = tid / CN;
  const int ntt = p.ntt, N3 = p.N3, Nt = p.Nt, h3 = N3 / 2;
  ColSmem<R> sm = col_carve<R>(smem, p, cw, false);
  col_twiddles(sm, p, tid, nth);
  __syncthreads();
  const int cidx = __builtin_amdgcn_readfirstlane(bx * (nth / CN) + cw);
  const bool live = cidx < ncol;
  const int cc = live ? cidx : 0;
  const int k2 = cc / p.J1, je = cc - k2 * p.J1;
  const size_t col = cc;
  double fac;
  int pol;
  column_policy(je, k2, p.N1, p.N2, fac, pol);
  const bool act = live && (SPEC || fac != 0.0);
  if (live && !act) {
    cpx<R>* z1 = static_cast<cpx<R>*>(out) + col * N3;
    for (int i = ct; i < N3; i += CN) z1[i] = cpx<R>{R(0), R(0)};
  }
  const cpx<R>* gc = G + col * Nt;
  // slot s of the padded line holds n' = s (s < ntt/2) or s - ntt; data index n = n' + Nt/2
  auto sample = [&](int s) {
    const int np = s < ntt / 2 ? s : s - ntt;
    const int n = np + Nt / 2;
    return (act && n >= 0 && n < Nt) ? gc[n] : cpx<R>{R(0), R(0)};
  };
  if (p.r_ntt.r[0] == 8 && ntt % 128 == 0) {
    // the first radix-8 stage straight from global memory: the samples go
    // from the loads into the butterflies, not through LDS first; the
    // stages keep the swizzled layout (swz) until the last, which writes
    // the plain one the gather reads
    stage_first_ip<8, (PPT + 7) / 8, true>(sm.a, ntt, ct, CN, sample);
    sync_policy<WV>();
    fft_lds_ip<false, R, WV, PPT, true>(sm.a, p.r_ntt, 1, 1, 0, col_twt(sm, p), ct, CN, 1, 8);
  } else {
    stage_in<(PPT < 16 ? PPT : 16)>(sm.a, ntt, ct, CN, sample);
    sync_policy<WV>();
    fft_lds_ip<false, R, WV, PPT>(sm.a, p.r_ntt, 1, 1, 0, col_twt(sm, p), ct, CN);
  }
  const cpx<R>* B = sm.a;
  if (ct < W) sm.a[ntt + ct] = sm.a[ct];
  sync_policy<WV>();
  const int j1 = je - p.N1 / 2;
  const double a = double(j1) * double(j1) * p.inv_L1sq + double(k2) * double(k2) * p.inv_L2sq;
  const double scale = SPEC ? p.scale_spec : p.scale_vol;
  const bool cosm = !SPEC && p.cosm != 0;
  const R cscale = R(scale);
  const R beta = R(p.beta);
  // Ratios of neighbouring window values: with d = o - fr,
  //   phi(o+1-fr) / phi(o-fr) = exp(-beta (2o+1)) exp(2 beta fr),
  // so one tap window needs three exponentials and a product chain running
  // out from the two taps nearest x; rk[k] = exp(-beta (2k+1)).
  R rk[W / 2];
#pragma unroll
  for (int k = 0; k < W / 2; ++k) rk[k] = R(exp(-p.beta * (2 * k + 1)));
  const bool chain = p.beta <= 8.0;  // exp(2 beta fr) stays far from overflow
  const R twow = R(2.0 / W);
  // the value of output li = ct + CN i, i < NLW, when they stay in registers
  cpx<R> hl[NLW];
  const bool in_regs = col_fl_in_regs(N3);
  // H(x) exp(-i phase) at the point lp
  auto taps = [&](const LPoint<R, ARGS64>& lp) {
    // taps q0 - W/2 + 1 .. q0 + W/2 read from b .. b + W - 1 (no wrap)
    const cpx<R>* Bq = B + pmodc(lp.q0 - W / 2 + 1, ntt) + (W / 2 - 1);
    cpx<R> H;
    if constexpr (KBW) {
      H = cpx<R>{R(0), R(0)};
#pragma unroll
      for (int o = -W / 2 + 1; o <= W / 2; ++o) H = H + Bq[o] * kb_tap<R>(R(o) - lp.fr, beta, twow);
    } else if (chain) {
      const R fr = lp.fr;
      const R up = wexp<R>(R(2) * beta * fr);
      const R dn = wexp<R>(R(-2) * beta * fr);
      const R phi0 = wexp<R>(-beta * fr * fr);
      H = Bq[0] * phi0;
      R ph = phi0;
#pragma unroll
      for (int o = 1; o <= W / 2; ++o) {
        ph = ph * (rk[o - 1] * up);
        H = H + Bq[o] * ph;
      }
      ph = phi0;
#pragma unroll
      for (int o = -1; o > -W / 2; --o) {
        ph = ph * (rk[-o - 1] * dn);
        H = H + Bq[o] * ph;
      }
    } else {
      H = cpx<R>{R(0), R(0)};
#pragma unroll
      for (int o = -W / 2 + 1; o <= W / 2; ++o) {
        const R d = R(o) - lp.fr;
        H = H + Bq[o] * wexp<R>(-beta * d * d);
      }
    }
    return cmul(H, lp.ph);
  };
  auto gather = [&](int li) {
    const LPoint<R, ARGS64> lp = lpoint<R, ARGS64>(p, a, li - h3, scale);
    return taps(lp) * (cosm ? cscale : lp.wgt);
  };
  if (in_regs) {
#pragma unroll
    for (int i = 0; i < NLW; ++i) {
      const int li = ct + CN * i;
      if (CN * i <= N3 && li <= N3) hl[i] = gather(li);
    }
  } else {
    for (int li = ct; li <= N3; li += CN) sm.fl[li] = gather(li);
  }
  // Q*: the l = 0 value from the two points +-x0
  cpx<R> hz = {R(0), R(0)};
  if (cosm && ct == 0) {
    const double x0 = x_lateral<ARGS64>(p, a);
    hz = (taps(lpoint_at<R, ARGS64>(p, x0)) + taps(lpoint_at<R, ARGS64>(p, -x0))) * (R(0.5) * cscale);
  }
  sync_policy<WV>();
  if constexpr (SPEC) {
    cpx<R>* F = static_cast<cpx<R>*>(out);
    const int N1 = p.N1, N2 = p.N2;
    // columns k2 in [0, N2/2) are written as they are (with N2 = 1 the one
    // row k2 = 0), the others through the Hermitian mirror
    const bool direct = act && k2 < (N2 + 1) / 2 && je < N1;
    const bool mirror = act && k2 >= 1 && je >= 1;
    const size_t rd = ((size_t)pmodc(j1, N1) * N2 + k2) * N3;
    const size_t rm = ((size_t)pmodc(-j1, N1) * N2 + pmodc(-k2, N2)) * N3;
    auto emit = [&](int li, cpx<R> v) {
      const int l = li - h3;
      if (direct && li < N3) F[rd + pmodc(l, N3)] = v;
      if (mirror && li > 0) F[rm + pmodc(-l, N3)] = conjg(v);
    };
    if (in_regs) {
#pragma unroll
      for (int i = 0; i < NLW; ++i) {
        const int li = ct + CN * i;
        if (CN * i <= N3 && li <= N3) emit(li, hl[i]);
      }
    } else {
      for (int li = ct; li <= N3; li += CN) emit(li, sm.fl[li]);
    }
  } else {
    // X[slot] for the depth inverse, in the transform buffer (free again):
    // slot (l mod N3) for |l| < N3/2; the two Nyquist representatives go to
    // slots N3/2 (l = -N3/2) and N3 (l = +N3/2) first and are combined after
    cpx<R>* X = sm.a;
    const R f = R(fac);
    auto place = [&](int li, cpx<R> v) {
      const int l = li - h3;
      const int s = li == N3 ? N3 : (l < 0 ? l + N3 : l);
      X[s] = v * f;
    };
    if (in_regs) {
#pragma unroll
      for (int i = 0; i < NLW; ++i) {
        const int li = ct + CN * i;
        if (CN * i <= N3 && li <= N3) place(li, hl[i]);
      }
    } else {
      for (int li = ct; li <= N3; li += CN) place(li, sm.fl[li]);
    }
    sync_policy<WV>();
    if (cosm) {
      // average slot s (l) with slot N3 - s (-l); the Nyquist pair is h3, N3;
      // slot 0 (l = 0) takes the two-point value
      if (ct == 0) X[0] = hz * f;
      for (int s = ct + 1; s < h3; s += CN) {
        const cpx<R> m = (X[s] + X[N3 - s]) * R(0.5);
        X[s] = m;
        X[N3 - s] = m;
      }
      if (ct == 0) {
        const cpx<R> m = (X[h3] + X[N3]) * R(0.5);
        X[h3] = m;
        X[N3] = m;
      }
      sync_policy<WV>();
    }
    if (ct == 0) {
      const cpx<R> lo = X[h3], hi = X[N3];
      X[h3] = pol == 0 ? lo : (pol == 1 ? hi : (lo + hi) * R(0.5));
    }
    sync_policy<WV>();
    fft_lds_ip<true, R, WV, PPT>(X, p.r_N3, 1, 1, 0, col_tw3(sm, p), ct, CN);
    const cpx<R>* Zr = X;
    if (act) {
      cpx<R>* z1 = static_cast<cpx<R>*>(out) + col * N3;
      for (int i = ct; i < N3; i += CN) z1[i] = Zr[i];
    }
  }
}

template <typename R, int W, bool ARGS64, bool SPEC, int PPT, bool KBW, int WPC>
__global__ __launch_bounds__(512) void k_column(KP p, int ncol, const cpx<R>* __restrict__ G, void* out) {
  column_body<R, W, ARGS64, SPEC, PPT, KBW, WPC>(p, ncol, blockIdx.x, G, out);
}

// First index i in [lo, hi) with q[i] >= v (q non-decreasing).
__device__ __forceinline__ int lower_bound_i(const int* q, int lo, int hi, int v) {
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (q[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

template <typename R, int W, bool ARGS64, int PPT, bool KBW, int WPC>
__device__ __forceinline__ void column_adj_body(const KP& p, int ncol, int mwrap, int bx,
                                                const cpx<R>* __restrict__ Z1, cpx<R>* __restrict__ G) {
  extern __shared__ __align__(16) char smem[];
  constexpr int CN = 64 * WPC;
  constexpr bool WV = WPC == 1;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int ct = tid % CN, cw = tid / CN;
  const int ntt = p.ntt, N3 = p.N3, Nt = p.Nt, h3 = N3 / 2;
  ColSmem<R> sm = col_carve<R>(smem, p, cw, true);
  col_twiddles(sm, p, tid, nth);
  __syncthreads();
  // a column past the end of the list, or one the half-spectrum inverse
  // leaves out, runs the same steps on zeros (every barrier is reached) and
  // writes only its zeros
  const int cidx = __builtin_amdgcn_readfirstlane(bx * (nth / CN) + cw);
  const bool live = cidx < ncol;
  const int cc = live ? cidx : 0;
  const int k2 = cc / p.J1, je = cc - k2 * p.J1;
  const size_t col = cc;
  double fac;
  int pol;
  column_policy(je, k2, p.N1, p.N2, fac, pol);
  const bool act = live && fac != 0.0;
  cpx<R>* gc = G + col * Nt;
  if (live && !act)
    for (int i = ct; i < Nt; i += CN) gc[i] = cpx<R>{R(0), R(0)};
  const cpx<R>* zc = Z1 + col * N3;
  stage_in<(PPT < 16 ? PPT : 16)>(sm.a, N3, ct, CN, [&](int i) { return act ? zc[i] : cpx<R>{R(0), R(0)}; });
  sync_policy<WV>();
  // transpose of the unnormalised depth inverse: forward FFT
  fft_lds_ip<false, R, WV, PPT>(sm.a, p.r_N3, 1, 1, 0, col_tw3(sm, p), ct, CN);
  const cpx<R>* Xp = sm.a;
  const int j1 = je - p.N1 / 2;
  const double a = double(j1) * double(j1) * p.inv_L1sq + double(k2) * double(k2) * p.inv_L2sq;
  const R f = R(fac);
  const R mlo = pol == 0 ? R(1) : (pol == 1 ? R(0) : R(0.5));
  const R mhi = pol == 1 ? R(1) : (pol == 0 ? R(0) : R(0.5));
  const bool cosm = p.cosm != 0;
  // F'(l) of output li: the Nyquist representatives share Xp[h3] by the policy
  auto fprime = [&](int li) {
    if (li == 0) return Xp[h3] * (f * mlo);
    if (li == N3) return Xp[h3] * (f * mhi);
    return Xp[pmodc(li - h3, N3)] * f;
  };
  // points e: output li = e; with cosm the l = 0 output is the pair of points
  // e = h3 (-x0) and h3 + 1 (+x0), and li = e - 1 above them
  const int npt = N3 + 1 + (cosm ? 1 : 0);
  const double x0 = cosm ? x_lateral<ARGS64>(p, a) : 0.0;
  for (int e = ct; e < npt; e += CN) {
    int li = e, side = 0;
    if (cosm && e >= h3) {
      if (e == h3)
        side = -1;
      else if (e == h3 + 1)
        li = h3, side = 1;
      else
        li = e - 1;
    }
    cpx<R> fp = fprime(li);
    LPoint<R, ARGS64> lp;
    if (cosm) {
      fp = (fp + fprime(N3 - li)) * R(0.5);  // transpose of the l, -l average
      lp = side ? lpoint_at<R, ARGS64>(p, side * x0) : lpoint<R, ARGS64>(p, a, li - h3, p.scale_vol);
      if (side) fp = fp * R(0.5);
      lp.wgt = R(p.scale_vol);
    } else {
      lp = lpoint<R, ARGS64>(p, a, li - h3, p.scale_vol);
    }
    sm.fl[e] = cmulc(fp, lp.ph) * lp.wgt;  // H'(l) = wgt * conj(ph) * F'(l)
    sm.q0[e] = lp.q0;
    sm.fr[e] = lp.fr;
  }
  sync_policy<WV>();
  // B'[q] = sum over l whose taps cover q of phi(x_l - q) H'(l); x_l is
  // non-decreasing in l, so the l covering q form a contiguous range.
  cpx<R>* Bp = sm.a;
  const R beta = R(p.beta);
  const R twow = R(2.0 / W);
  // the points' grid cells span [qlo, qhi]; an image of the time grid whose
  // tap window misses that span has no contribution
  const int qlo = sm.q0[0], qhi = sm.q0[npt - 1];
  // st[v] = number of points with q0 < qlo + v (v in [0, span + 1]). The
  // points' cells q0 are non-decreasing, so st[v] = e for the cells v in
  // (q0[e-1] - qlo, q0[e] - qlo]: each lane fills the cells between its
  // point and the one before (no atomics, no scan), 16-bit entries (npt <=
  // 4098). The bounds of a tap window are then single reads. A span beyond
  // the table (aliased frequencies) keeps the binary search.
  const int span = qhi - qlo;
  const bool table = span <= ntt;
  short* st = sm.st;
  if (table) {
    for (int e = ct; e < npt; e += CN) {
      const int hv = sm.q0[e] - qlo;
      const int lv = e == 0 ? 0 : sm.q0[e - 1] - qlo + 1;
      for (int v = lv; v <= hv; ++v) st[v] = short(e);
    }
    if (ct == 0) st[span + 1] = short(npt);
    sync_policy<WV>();
  }
  // first point with q0 >= t
  auto lower = [&](int t, int from) {
    if (!table) return lower_bound_i(sm.q0, from, npt, t);
    const int v = t - qlo;
    return v <= 0 ? 0 : (v > span ? npt : int(st[v]));
  };
  // the transform buffer is not read here (the loop reads the per-point
  // arrays and the table), so each B' value goes straight into it
  for (int q = ct; q < ntt; q += CN) {
    const int qc = q < ntt / 2 ? q : q - ntt;
    cpx<R> acc = {R(0), R(0)};
    for (int m = -mwrap; m <= mwrap; ++m) {
      const int qv = qc + m * ntt;
      if (qv + W / 2 - 1 < qlo || qv - W / 2 > qhi) continue;
      // tap o = qv - q0 must lie in [-W/2+1, W/2]: q0 in [qv - W/2, qv + W/2 - 1]
      const int lo = lower(qv - W / 2, 0);
      const int hi = lower(qv + W / 2, lo);
      for (int li = lo; li < hi; ++li) {
        const R d = R(qv - sm.q0[li]) - sm.fr[li];
        if constexpr (KBW)
          acc = acc + sm.fl[li] * kb_tap<R>(d, beta, twow);
        else
          acc = acc + sm.fl[li] * wexp<R>(-beta * d * d);
      }
    }
    Bp[q] = acc;
  }
  sync_policy<WV>();
  fft_lds_ip<true, R, WV, PPT>(Bp, p.r_ntt, 1, 1, 0, col_twt(sm, p), ct, CN);
  const cpx<R>* Ap = Bp;
  if (act) {
    for (int n = ct; n < Nt; n += CN) {
      const int s = pmodc(n - Nt / 2, ntt);
      gc[n] = Ap[s];
    }
  }
}

template <typename R, int W, bool ARGS64, int PPT, bool KBW, int WPC>
__global__ __launch_bounds__(512) void k_column_adj(KP p, int ncol, int mwrap, const cpx<R>* __restrict__ Z1,
                                                    cpx<R>* __restrict__ G) {
  column_adj_body<R, W, ARGS64, PPT, KBW, WPC>(p, ncol, mwrap, blockIdx.x, Z1, G);
}

// ---------------------------------------------------------------- launchers

// Columns per workgroup (up to 512 threads): the count that keeps the most
// wavefronts resident on a CU with 160 KB of LDS (the twiddles are shared).
template <typename R>
static int cols_per_wg(const KP& p, bool adj, int wpc) {
  const size_t sh = col_shared_bytes<R>(p.ntt, p.N3), per = col_wave_bytes<R>(p.ntt, p.N3, adj);
  const size_t lds = 160 * 1024;
  int best = 1;
  size_t best_waves = 0;
  for (int c = 1; c * wpc <= 8; ++c) {
    const size_t wg = sh + c * per;
    if (wg > lds) break;
    const size_t waves = c * wpc * (lds / wg);
    if (waves > best_waves) {
      best_waves = waves;
      best = c;
    }
  }
  return best;
}

// Points per thread of the per-column transforms: the larger of ntt and N3
// over the column's threads, rounded up to a power of two (at least 4).
static int column_ppt(const KP& p) {
  const int n = p.ntt > p.N3 ? p.ntt : p.N3;
  const int need = (n + 64 * column_wpc(p.ntt, p.N3) - 1) / (64 * column_wpc(p.ntt, p.N3));
  return need <= 4 ? 4 : need <= 8 ? 8 : 16;
}

template <typename R, int W, bool ARGS64, int PPT, bool KBW, int WPC>
static hipError_t column_wp(const KP& p, const void* G, void* out, int spec, hipStream_t s) {
  const int cpw = cols_per_wg<R>(p, false, WPC);
  const int ncol = p.J1 * p.K2;
  const size_t sh = col_shared_bytes<R>(p.ntt, p.N3) + cpw * col_wave_bytes<R>(p.ntt, p.N3, false);
  dim3 grid((ncol + cpw - 1) / cpw);
  hipError_t e = allow_smem(spec ? k_column<R, W, ARGS64, true, PPT, KBW, WPC>
                                 : k_column<R, W, ARGS64, false, PPT, KBW, WPC>, sh);
  if (e != hipSuccess) return e;
  if (spec)
    hipLaunchKernelGGL((k_column<R, W, ARGS64, true, PPT, KBW, WPC>), grid, dim3(64 * WPC * cpw), sh, s, p, ncol,
                       static_cast<const cpx<R>*>(G), out);
  else
    hipLaunchKernelGGL((k_column<R, W, ARGS64, false, PPT, KBW, WPC>), grid, dim3(64 * WPC * cpw), sh, s, p,
                       ncol, static_cast<const cpx<R>*>(G), out);
  return hipGetLastError();
}

template <typename R, int W, bool ARGS64, int PPT, bool KBW, int WPC>
static hipError_t column_adj_wp(const KP& p, const void* Z1, void* G, hipStream_t s) {
  const int cpw = cols_per_wg<R>(p, true, WPC);
  const int ncol = p.J1 * p.K2;
  const size_t sh = col_shared_bytes<R>(p.ntt, p.N3) + cpw * col_wave_bytes<R>(p.ntt, p.N3, true);
  dim3 grid((ncol + cpw - 1) / cpw);
  // number of periodic images of the time grid a tap window can reach
  const double xmax = p.cdtnt * sqrt((p.N1 / 2.0) * (p.N1 / 2.0) * p.inv_L1sq +
                                     (p.N2 / 2.0) * (p.N2 / 2.0) * p.inv_L2sq +
                                     (p.N3 / 2.0) * (p.N3 / 2.0) * p.bz);
  const int mwrap = 1 + int((xmax + W) / p.ntt);
  hipError_t e = allow_smem(k_column_adj<R, W, ARGS64, PPT, KBW, WPC>, sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_column_adj<R, W, ARGS64, PPT, KBW, WPC>), grid, dim3(64 * WPC * cpw), sh, s, p, ncol,
                     mwrap, static_cast<const cpx<R>*>(Z1), static_cast<cpx<R>*>(G));
  return hipGetLastError();
}

// (wavefronts per column, points per thread): (1, 4), (1, 8) up to 512
// points, (4, 4), (4, 8), (4, 16) up to 4096
template <typename R, int W, bool ARGS64, bool KBW>
static hipError_t column_w(const KP& p, const void* G, void* out, int spec, hipStream_t s) {
  const int ppt = column_ppt(p);
  if (column_wpc(p.ntt, p.N3) == 1)
    return ppt == 4 ? column_wp<R, W, ARGS64, 4, KBW, 1>(p, G, out, spec, s)
                    : column_wp<R, W, ARGS64, 8, KBW, 1>(p, G, out, spec, s);
  return ppt == 4 ? column_wp<R, W, ARGS64, 4, KBW, 4>(p, G, out, spec, s)
                  : ppt == 8 ? column_wp<R, W, ARGS64, 8, KBW, 4>(p, G, out, spec, s)
                             : column_wp<R, W, ARGS64, 16, KBW, 4>(p, G, out, spec, s);
}

template <typename R, int W, bool ARGS64, bool KBW>
static hipError_t column_adj_w(const KP& p, const void* Z1, void* G, hipStream_t s) {
  const int ppt = column_ppt(p);
  if (column_wpc(p.ntt, p.N3) == 1)
    return ppt == 4 ? column_adj_wp<R, W, ARGS64, 4, KBW, 1>(p, Z1, G, s)
                    : column_adj_wp<R, W, ARGS64, 8, KBW, 1>(p, Z1, G, s);
  return ppt == 4 ? column_adj_wp<R, W, ARGS64, 4, KBW, 4>(p, Z1, G, s)
                  : ppt == 8 ? column_adj_wp<R, W, ARGS64, 8, KBW, 4>(p, Z1, G, s)
                             : column_adj_wp<R, W, ARGS64, 16, KBW, 4>(p, Z1, G, s);
}

// The Kaiser-Bessel window is instantiated for the tap counts it is meant
// for (4 to 12); the descriptor check rejects the others.
constexpr bool kb_width(int W) { return W >= 4 && W <= 12; }

template <typename R, bool ARGS64>
hipError_t column_a(const KP& p, const void* in, void* out, int spec, hipStream_t s, bool adj) {
  switch (p.W) {
#define NEDNER_CW(WV)                                                                                   \
  case WV:                                                                                             \
    if constexpr (kb_width(WV)) {                                                                      \
      if (p.window == 1)                                                                               \
        return adj ? column_adj_w<R, WV, ARGS64, true>(p, in, out, s)                                  \
                   : column_w<R, WV, ARGS64, true>(p, in, out, spec, s);                               \
    }                                                                                                  \
    if (p.window != 0) return hipErrorInvalidValue;                                                    \
    return adj ? column_adj_w<R, WV, ARGS64, false>(p, in, out, s) : column_w<R, WV, ARGS64, false>(p, in, out, spec, s);
    NEDNER_CW(2)
    NEDNER_CW(4)
    NEDNER_CW(6)
    NEDNER_CW(8)
    NEDNER_CW(10)
    NEDNER_CW(12)
    NEDNER_CW(14)
    NEDNER_CW(16)
#undef NEDNER_CW
    default:
      return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------- batched
template <typename R, int W, bool ARGS64, int PPT, bool KBW, int WPC>
__global__ __launch_bounds__(512) void k_column_many(const BatchProb* __restrict__ bp, WorkList wl) {
  work_loop(wl, [&](int prob, int local) {
    const BatchProb& B = bp[prob];
    const KP& p = B.kp;
    column_body<R, W, ARGS64, false, PPT, KBW, WPC>(p, p.J1 * p.K2, local, static_cast<const cpx<R>*>(B.b0),
                                                    B.b1);
  });
}

template <typename R, int W, bool ARGS64, int PPT, bool KBW, int WPC>
static hipError_t column_many_wp(const BatchProb* bp, const WorkList& wl, int cpw, size_t smem, hipStream_t s) {
  if (wl.total <= 0) return hipSuccess;
  auto k = k_column_many<R, W, ARGS64, PPT, KBW, WPC>;
  hipError_t e = allow_smem(k, smem);
  if (e != hipSuccess) return e;
  int per_cu = 0, dev = 0, cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), 64 * WPC * cpw,
                                                   smem) != hipSuccess || per_cu < 1)
    per_cu = 1;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int grid = (int)std::min<long>((long)per_cu * cus, wl.total);
  hipLaunchKernelGGL(k, dim3(grid), dim3(64 * WPC * cpw), smem, s, bp, wl);
  return hipGetLastError();
}

// p0 carries the largest ntt and N3 of the batch: they fix the wavefronts per
// column and the points per thread of the launch
template <typename R, bool ARGS64>
hipError_t column_many_a(const KP& p0, int ppt, const BatchProb* bp, const WorkList& wl, int cpw,
                                size_t smem, hipStream_t s) {
  const int wpc = column_wpc(p0.ntt, p0.N3);
#define NEDNER_CMPK(WV, KB)                                                                        \
    if (wpc == 1)                                                                                  \
      return ppt == 4 ? column_many_wp<R, WV, ARGS64, 4, KB, 1>(bp, wl, cpw, smem, s)              \
                      : column_many_wp<R, WV, ARGS64, 8, KB, 1>(bp, wl, cpw, smem, s);             \
    return ppt == 4 ? column_many_wp<R, WV, ARGS64, 4, KB, 4>(bp, wl, cpw, smem, s)                \
                    : ppt == 8 ? column_many_wp<R, WV, ARGS64, 8, KB, 4>(bp, wl, cpw, smem, s)     \
                               : column_many_wp<R, WV, ARGS64, 16, KB, 4>(bp, wl, cpw, smem, s);
#define NEDNER_CMP(WV)                                                                   \
  case WV:                                                                               \
    if constexpr (kb_width(WV)) {                                                        \
      if (p0.window == 1) { NEDNER_CMPK(WV, true) }                                      \
    }                                                                                    \
    if (p0.window != 0) return hipErrorInvalidValue;                                     \
    NEDNER_CMPK(WV, false)
  switch (p0.W) {
    NEDNER_CMP(2)
    NEDNER_CMP(4)
    NEDNER_CMP(6)
    NEDNER_CMP(8)
    NEDNER_CMP(10)
    NEDNER_CMP(12)
    NEDNER_CMP(14)
    NEDNER_CMP(16)
    default: return hipErrorInvalidValue;
  }
#undef NEDNER_CMP
#undef NEDNER_CMPK
}

}  // namespace nedner

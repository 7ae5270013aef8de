// Mixed-radix Stockham FFT staged in LDS for gfx950.
//
// A workgroup transforms `lines` independent lines of length n held in LDS.
// Point p of line b sits at buf[p * ps + b * ls]. Each stage reads one LDS
// buffer and writes the other (ping-pong), so one barrier per stage suffices;
// the result ends in the buffer selected by the parity of the stage count.
// Radices 2, 3, 4, 5 and 8 cover every 5-smooth length. Twiddles come from a
// table tw[k] = exp(-2 pi i k / n) computed in double on the host and staged
// in LDS by the caller.
#pragma once
#include <hip/hip_runtime.h>

namespace nedner {

template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T x, T y) { return cpx<T>{x, y}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> conjg(cpx<T> a) { return {a.x, -a.y}; }
// multiply by -i (forward kernels) or +i (inverse kernels)
template <bool INV, typename T>
__device__ __forceinline__ cpx<T> rot(cpx<T> a) {
  return INV ? cpx<T>{-a.y, a.x} : cpx<T>{a.y, -a.x};
}

// Radix sequence of one transform length, chosen on the host.
struct Radices {
  int n;
  int count;
  int r[16];
};

// Twiddle lookup: a full table tw[i] = exp(-2 pi i / n) (a plain pointer), or
// the first half of one (TwHalf: tw[i + n/2] = -tw[i]) read at index i * mul,
// so that a length-n/mul transform can use the table of a length-n one.
template <typename T>
struct TwHalf {
  const cpx<T>* t;
  int mul;  // index stride into the table
  int nh;   // entries held: half the table's length
};
// twstride: the factor an exponent i is scaled by into the table; twat: the
// entry at an index already scaled (one lookup, the sign of the second half
// applied by selects rather than a branch per lane).
template <typename T>
__device__ __forceinline__ int twstride(const cpx<T>*) { return 1; }
template <typename T>
__device__ __forceinline__ int twstride(const TwHalf<T>& tw) { return tw.mul; }
template <typename T>
__device__ __forceinline__ cpx<T> twat(const cpx<T>* tw, int ii) { return tw[ii]; }
template <typename T>
__device__ __forceinline__ cpx<T> twat(const TwHalf<T>& tw, int ii) {
  const bool up = ii >= tw.nh;
  const cpx<T> w = tw.t[up ? ii - tw.nh : ii];
  return cpx<T>{up ? -w.x : w.x, up ? -w.y : w.y};
}
template <typename T>
__device__ __forceinline__ cpx<T> twget(const cpx<T>* tw, int i) { return tw[i]; }
template <typename T>
__device__ __forceinline__ cpx<T> twget(const TwHalf<T>& tw, int i) { return twat(tw, i * tw.mul); }

template <int R, bool INV, typename T>
__device__ __forceinline__ void dft_small(cpx<T>* v) {
  if constexpr (R == 2) {
    cpx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 3) {
    const T h = T(0.8660254037844386467637231707529362);
    cpx<T> t1 = v[1] + v[2];
    cpx<T> t2 = v[0] - t1 * T(0.5);
    cpx<T> t3 = (v[1] - v[2]) * h;
    v[0] = v[0] + t1;
    cpx<T> r3 = rot<INV>(t3);
    v[1] = t2 + r3;
    v[2] = t2 - r3;
  } else if constexpr (R == 4) {
    cpx<T> a = v[0] + v[2], b = v[0] - v[2];
    cpx<T> c = v[1] + v[3], d = rot<INV>(v[1] - v[3]);
    v[0] = a + c;
    v[2] = a - c;
    v[1] = b + d;
    v[3] = b - d;
  } else if constexpr (R == 5) {
    const T c1 = T(0.3090169943749474241022934171828191);
    const T c2 = T(-0.8090169943749474241022934171828191);
    const T s1 = T(0.9510565162951535721164393333793821);
    const T s2 = T(0.5877852522924731291687059546390728);
    cpx<T> t1 = v[1] + v[4], t2 = v[2] + v[3];
    cpx<T> t3 = v[1] - v[4], t4 = v[2] - v[3];
    cpx<T> a1 = v[0] + t1 * c1 + t2 * c2;
    cpx<T> a2 = v[0] + t1 * c2 + t2 * c1;
    cpx<T> b1 = rot<INV>(t3 * s1 + t4 * s2);
    cpx<T> b2 = rot<INV>(t3 * s2 - t4 * s1);
    v[0] = v[0] + t1 + t2;
    v[1] = a1 + b1;
    v[4] = a1 - b1;
    v[2] = a2 + b2;
    v[3] = a2 - b2;
  } else if constexpr (R == 8) {
    const T q = T(0.7071067811865475244008443621048490);
    cpx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cpx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft_small<4, INV>(e);
    dft_small<4, INV>(o);
    // twiddles exp(-+ 2 pi i k / 8), k = 1..3
    cpx<T> o1 = cpx<T>{(o[1].x + (INV ? -o[1].y : o[1].y)) * q, (o[1].y + (INV ? o[1].x : -o[1].x)) * q};
    cpx<T> o2 = rot<INV>(o[2]);
    cpx<T> o3 = cpx<T>{(-o[3].x + (INV ? -o[3].y : o[3].y)) * q,
                       (-o[3].y + (INV ? o[3].x : -o[3].x)) * q};
    v[0] = e[0] + o[0];
    v[4] = e[0] - o[0];
    v[1] = e[1] + o1;
    v[5] = e[1] - o1;
    v[2] = e[2] + o2;
    v[6] = e[2] - o2;
    v[3] = e[3] + o3;
    v[7] = e[3] - o3;
  }
}

// One Stockham stage of radix R over all lines: src -> dst.
template <int R, bool INV, typename T>
__device__ __forceinline__ void stockham_stage(const cpx<T>* __restrict__ src, cpx<T>* __restrict__ dst,
                                               int n, int Ns, int lines, int ps, int ls,
                                               const cpx<T>* __restrict__ tw, int tid, int nth) {
  const int nb = n / R;
  const int total = nb * lines;
  const int tstep = n / (Ns * R);
  for (int t = tid; t < total; t += nth) {
    const int b = t % lines;
    const int j = t / lines;
    const int k = j % Ns;
    cpx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[(j + r * nb) * ps + b * ls];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cpx<T> w = tw[r * k * tstep];
        v[r] = INV ? cmulc(v[r], w) : cmul(v[r], w);
      }
    }
    dft_small<R, INV>(v);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(base + r * Ns) * ps + b * ls] = v[r];
  }
}

// Make this wavefront's LDS writes visible to its own later LDS reads.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Full transform. Returns the buffer holding the result (a or b). Caller must
// synchronise before the call (data in `a` visible); on return the result is
// visible to every thread that took part. WAVE: the transform is done by one
// wavefront alone (tid = lane, nth = 64) and only waits on its own LDS traffic.
template <bool INV, typename T, bool WAVE = false>
__device__ cpx<T>* fft_lds(cpx<T>* a, cpx<T>* b, const Radices& rd, int lines, int ps, int ls,
                           const cpx<T>* tw, int tid, int nth) {
  int Ns = 1;
  for (int s = 0; s < rd.count; ++s) {
    const int R = rd.r[s];
    switch (R) {
      case 2: stockham_stage<2, INV>(a, b, rd.n, Ns, lines, ps, ls, tw, tid, nth); break;
      case 3: stockham_stage<3, INV>(a, b, rd.n, Ns, lines, ps, ls, tw, tid, nth); break;
      case 4: stockham_stage<4, INV>(a, b, rd.n, Ns, lines, ps, ls, tw, tid, nth); break;
      case 5: stockham_stage<5, INV>(a, b, rd.n, Ns, lines, ps, ls, tw, tid, nth); break;
      default: stockham_stage<8, INV>(a, b, rd.n, Ns, lines, ps, ls, tw, tid, nth); break;
    }
    if constexpr (WAVE)
      wave_sync();
    else
      __syncthreads();
    cpx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// In-place variant for a whole workgroup: each stage first gathers the inputs
// of all of a thread's butterflies into registers, then (after a barrier)
// writes the outputs over the same buffer. Half the LDS of the ping-pong form,
// at the price of a second barrier per stage. K is the number of butterflies
// a thread handles per stage (K * nth >= butterflies of the stage).
template <bool WAVE>
__device__ __forceinline__ void sync_policy() {
  if constexpr (WAVE)
    wave_sync();
  else
    __syncthreads();
}

// Swizzled layout of a single line (lines = 1, ps = 1): point i at
// i ^ ((i >> 4) & 7), a permutation within each block of 16 points (128
// bytes of complex float: the 32 LDS banks). The first radix-8 stage writes
// each butterfly's outputs to 8 consecutive points, so the lanes of a
// wavefront write 64 bytes apart: in the plain layout 16 lanes fall on the
// same 2 bank pairs (an 8-way conflict); the swizzle gives each of them its
// own pair, and 16 consecutive points aligned to 16 stay on 16 distinct pairs.
// The footprint is unchanged (no LDS is added).
__device__ __forceinline__ int swz(int i) { return i ^ ((i >> 4) & 7); }

// `lines` is a power of two; Ns (the product of the radices already done) is
// one for power-of-two lengths, so the index arithmetic is shifts and masks
// there and true divisions only for lengths with factors 3 or 5.
// PIN, POUT: the stage reads / writes the swizzled layout (single lines only).
template <int R, int K, bool INV, typename T, bool WAVE = false, bool PIN = false, bool POUT = false,
          typename TWT = const cpx<T>*>
__device__ __forceinline__ void stage_ip(cpx<T>* buf, int n, int Ns, int lines, int ps, int ls,
                                         const TWT& tw, int tid, int nth) {
  const int nb = n / R;
  const int total = nb * lines;
  const int tstep = n / (Ns * R);
  const int lsh = __builtin_ctz(lines);
  const bool ns_pow2 = (Ns & (Ns - 1)) == 0;
  cpx<T> v[K][R];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int t = tid + q * nth;
    if (t < total) {
      const int b = t & (lines - 1), j = t >> lsh;
#pragma unroll
      for (int r = 0; r < R; ++r)
        v[q][r] = PIN ? buf[swz(j + r * nb)] : buf[(j + r * nb) * ps + b * ls];
    }
  }
  sync_policy<WAVE>();
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int t = tid + q * nth;
    if (t < total) {
      const int b = t & (lines - 1), j = t >> lsh;
      const int k = ns_pow2 ? (j & (Ns - 1)) : (j % Ns);
      if (Ns > 1) {
        // exponent r k tstep, scaled into the table once per butterfly
        const int kt = k * (tstep * twstride(tw));
#pragma unroll
        for (int r = 1; r < R; ++r) {
          cpx<T> w = twat(tw, r * kt);
          v[q][r] = INV ? cmulc(v[q][r], w) : cmul(v[q][r], w);
        }
      }
      dft_small<R, INV>(v[q]);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (POUT)
          buf[swz(base + r * Ns)] = v[q][r];
        else
          buf[(base + r * Ns) * ps + b * ls] = v[q][r];
      }
    }
  }
  sync_policy<WAVE>();
}

// Whole transform in place. PPT bounds the points per thread (n * lines <=
// PPT * nth), which fixes the register array of every stage at compile time:
// a thread holds ceil(PPT / R) butterflies of radix R. Caller synchronises
// before; the result is in `buf` and visible on return.
// s0, Ns0: start at stage s0 with Ns0 the product of the radices before it
// (the earlier stages done by the caller, see stage_first_ip).
// PAD (single lines only): the line arrives in the swizzled layout and every
// stage but the last keeps it; the last writes the plain layout.
// Always inlined: as a called function its per-stage register arrays would
// live in scratch memory (the compiler declines to inline it into the
// largest column kernels otherwise).
template <bool INV, typename T, bool WAVE, int PPT, bool PAD = false, typename TWT = const cpx<T>*>
__device__ __forceinline__ void fft_lds_ip(cpx<T>* buf, const Radices& rd, int lines, int ps, int ls, const TWT& tw,
                           int tid, int nth, int s0 = 0, int Ns0 = 1) {
  int Ns = Ns0;
  for (int s = s0; s < rd.count; ++s) {
    const int R = rd.r[s];
    const bool last = s + 1 == rd.count;
#define NEDNER_STAGE(RR)                                                                                  \
  if (PAD && !last)                                                                                       \
    stage_ip<RR, (PPT + RR - 1) / RR, INV, T, WAVE, PAD, PAD, TWT>(buf, rd.n, Ns, lines, ps, ls, tw, tid,    \
                                                                  nth);                                   \
  else                                                                                                    \
    stage_ip<RR, (PPT + RR - 1) / RR, INV, T, WAVE, PAD, false, TWT>(buf, rd.n, Ns, lines, ps, ls, tw, tid,  \
                                                                    nth);
    switch (R) {
      case 2: NEDNER_STAGE(2) break;
      case 3: NEDNER_STAGE(3) break;
      case 4: NEDNER_STAGE(4) break;
      case 5: NEDNER_STAGE(5) break;
      default: NEDNER_STAGE(8) break;
    }
#undef NEDNER_STAGE
    Ns *= R;
  }
}

// The first Stockham stage (Ns = 1) of a single line of length n with radix
// R, its inputs taken from f(i) (typically global loads) instead of LDS: the
// line never has to be staged in LDS before the transform. Butterfly j reads
// points j + r n/R, r < R, and writes its outputs to point j R + r (of the
// swizzled layout with POUT). K butterflies per thread (K * nth >= n / R). The
// caller synchronises after.
template <int R, int K, bool POUT, typename T, typename F>
__device__ __forceinline__ void stage_first_ip(cpx<T>* buf, int n, int tid, int nth, F&& f) {
  const int nb = n / R;
  cpx<T> v[K][R];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int j = tid + q * nth;
#pragma unroll
    for (int r = 0; r < R; ++r) v[q][r] = j < nb ? f(j + r * nb) : cpx<T>{T(0), T(0)};
  }
#pragma unroll
  for (int q = 0; q < K; ++q) {
    const int j = tid + q * nth;
    if (j < nb) {
      dft_small<R, false>(v[q]);
#pragma unroll
      for (int r = 0; r < R; ++r) buf[POUT ? swz(j * R + r) : j * R + r] = v[q][r];
    }
  }
}

// Fill dst[0, total) with f(i) (each f typically one global load), thread tid
// of nth taking i = tid, tid + nth, ... . Up to BATCH loads per thread are in
// flight before the first LDS store, so their latencies overlap instead of
// adding up as they do when every store waits for its own load.
template <int BATCH, typename T, typename F>
__device__ __forceinline__ void stage_in(cpx<T>* dst, int total, int tid, int nth, F&& f) {
  for (int base = 0; base < total; base += BATCH * nth) {
    cpx<T> v[BATCH];
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int i = base + tid + q * nth;
      v[q] = i < total ? f(i) : cpx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int i = base + tid + q * nth;
      if (i < total) dst[i] = v[q];
    }
  }
}

// Stage a twiddle table of n entries from global memory into LDS.
template <typename T>
__device__ __forceinline__ void load_twiddles(cpx<T>* dst, const cpx<T>* __restrict__ src, int n,
                                              int tid, int nth) {
  for (int i = tid; i < n; i += nth) dst[i] = src[i];
}

}  // namespace nedner

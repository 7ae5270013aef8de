// Host-side dispatch of the spreading (eq. (10)) and sensor-gather kernels
// (k_spread_impl.hpp) over the precisions, each instantiated in a translation
// unit of its own; the batch preparation kernel; the equispaced placement.
#include "k_spread_impl.hpp"

namespace nedner {

extern template hipError_t spread_p<double, double, double, false>(const KP&, const void*, void*, int, hipStream_t, bool);
extern template hipError_t spread_many_p<double, double, double, false>(const KP&, const BatchProb*, const WorkList&, bool,
                                                      hipStream_t);
extern template int occ_p<double, double, double, false>(const KP&);
extern template hipError_t spread_p<float, float, float, false>(const KP&, const void*, void*, int, hipStream_t, bool);
extern template hipError_t spread_many_p<float, float, float, false>(const KP&, const BatchProb*, const WorkList&, bool,
                                                      hipStream_t);
extern template int occ_p<float, float, float, false>(const KP&);
extern template hipError_t spread_p<float, float, float, true>(const KP&, const void*, void*, int, hipStream_t, bool);
extern template hipError_t spread_many_p<float, float, float, true>(const KP&, const BatchProb*, const WorkList&, bool,
                                                      hipStream_t);
extern template int occ_p<float, float, float, true>(const KP&);
extern template hipError_t spread_p<float, double, double, false>(const KP&, const void*, void*, int, hipStream_t, bool);
extern template hipError_t spread_many_p<float, double, double, false>(const KP&, const BatchProb*, const WorkList&, bool,
                                                      hipStream_t);
extern template int occ_p<float, double, double, false>(const KP&);
extern template hipError_t spread_p<float, float, double, false>(const KP&, const void*, void*, int, hipStream_t, bool);
extern template hipError_t spread_many_p<float, float, double, false>(const KP&, const BatchProb*, const WorkList&, bool,
                                                      hipStream_t);
extern template int occ_p<float, float, double, false>(const KP&);

static int vec_ok(const KP& p, const void* a, const void* b, size_t esz) {
  const size_t al = (size_t)p.TT * esz;
  if (p.Nt % p.TT) return 0;
  if (((uintptr_t)a % al) || ((uintptr_t)b % al)) return 0;
  return 1;
}

// Element, weight and accumulation types of each precision: FP64 double
// throughout; FP32W float data with double sums and (by default) double
// first-axis weights; FP32C float with Kahan-compensated float sums; FP32 and
// FP32P float.
static hipError_t dispatch(const KP& p, const void* a, void* b, hipStream_t s, bool adj) {
  switch (p.prec) {
    case PREC_FP64: return spread_p<double, double, double, false>(p, a, b, vec_ok(p, a, b, 8), s, adj);
    case PREC_FP32W:
      return p.wide_w ? spread_p<float, double, double, false>(p, a, b, vec_ok(p, a, b, 4), s, adj)
                      : spread_p<float, float, double, false>(p, a, b, vec_ok(p, a, b, 4), s, adj);
    case PREC_FP32C: return spread_p<float, float, float, true>(p, a, b, vec_ok(p, a, b, 4), s, adj);
    default: return spread_p<float, float, float, false>(p, a, b, vec_ok(p, a, b, 4), s, adj);
  }
}

__global__ void k_batch_prepare(BatchProb* bp, PtrChunk c, int* counters, int ncounters) {
  const int i = threadIdx.x;
  if (i < c.n) {
    bp[c.first + i].g = c.g[i];
    bp[c.first + i].out = c.out[i];
  }
  if (i < ncounters) counters[i] = 0;
}

hipError_t launch_batch_prepare(BatchProb* bp, const PtrChunk& c, int* counters, int ncounters,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_batch_prepare, dim3(1), dim3(64), 0, s, bp, c, counters, ncounters);
  return hipGetLastError();
}

hipError_t launch_spread_many(const KP& p0, const BatchProb* bp, const WorkList& wl, int vec,
                              hipStream_t s) {
  switch (p0.prec) {
    case PREC_FP64: return spread_many_p<double, double, double, false>(p0, bp, wl, vec != 0, s);
    case PREC_FP32W:
      return p0.wide_w ? spread_many_p<float, double, double, false>(p0, bp, wl, vec != 0, s)
                       : spread_many_p<float, float, double, false>(p0, bp, wl, vec != 0, s);
    case PREC_FP32C: return spread_many_p<float, float, float, true>(p0, bp, wl, vec != 0, s);
    default: return spread_many_p<float, float, float, false>(p0, bp, wl, vec != 0, s);
  }
}

// ---------------------------------------------------------------------------
// Sensors on the output grid (the equispaced, NER-only case): the lateral
// sums of eq. (5) are a plain DFT of the node grid, so the spreading becomes
// a placement, U[q1][q2][n] = s_m g[m][n] at the sensor's node and zero at
// the other nodes, and its transpose a pick-up. One workgroup per (node or
// sensor, 256 samples), coalesced along time.

template <typename R>
__global__ __launch_bounds__(256) void k_place(KP p, int tchunks, const R* __restrict__ g, R* __restrict__ U) {
  const long nd = blockIdx.x / tchunks;
  const int t = (blockIdx.x % tchunks) * 256 + threadIdx.x;
  if (t >= p.Nt) return;
  const int m = p.node[nd];
  U[nd * p.Nt + t] = m >= 0 ? static_cast<const R*>(p.sw)[m] * g[(size_t)m * p.Nt + t] : R(0);
}

template <typename R>
__global__ __launch_bounds__(256) void k_place_adj(KP p, int tchunks, const R* __restrict__ U, R* __restrict__ g) {
  const long m = blockIdx.x / tchunks;
  const int t = (blockIdx.x % tchunks) * 256 + threadIdx.x;
  if (t >= p.Nt) return;
  const size_t nd = (size_t)p.cell[2 * m] * p.n2 + p.cell[2 * m + 1];
  g[m * p.Nt + t] = static_cast<const R*>(p.sw)[m] * U[nd * p.Nt + t];
}

hipError_t launch_place(const KP& p, const void* g, void* U, hipStream_t s) {
  const int tch = (p.Nt + 255) / 256;
  const dim3 grid((unsigned)((long)p.n1 * p.n2 * tch));
  if (p.prec == PREC_FP64)
    hipLaunchKernelGGL(k_place<double>, grid, dim3(256), 0, s, p, tch, static_cast<const double*>(g),
                       static_cast<double*>(U));
  else
    hipLaunchKernelGGL(k_place<float>, grid, dim3(256), 0, s, p, tch, static_cast<const float*>(g),
                       static_cast<float*>(U));
  return hipGetLastError();
}

hipError_t launch_place_adj(const KP& p, const void* U, void* g, hipStream_t s) {
  const int tch = (p.Nt + 255) / 256;
  const dim3 grid((unsigned)((long)p.M * tch));
  if (p.prec == PREC_FP64)
    hipLaunchKernelGGL(k_place_adj<double>, grid, dim3(256), 0, s, p, tch, static_cast<const double*>(U),
                       static_cast<double*>(g));
  else
    hipLaunchKernelGGL(k_place_adj<float>, grid, dim3(256), 0, s, p, tch, static_cast<const float*>(U),
                       static_cast<float*>(g));
  return hipGetLastError();
}

int spread_blocks_per_cu(const KP& p) {
  switch (p.prec) {
    case PREC_FP64: return occ_p<double, double, double, false>(p);
    case PREC_FP32W: return p.wide_w ? occ_p<float, double, double, false>(p) : occ_p<float, float, double, false>(p);
    case PREC_FP32C: return occ_p<float, float, float, true>(p);
    default: return occ_p<float, float, float, false>(p);
  }
}

hipError_t launch_spread(const KP& p, const void* g, void* U, hipStream_t s) {
  return dispatch(p, g, U, s, false);
}

hipError_t launch_gather(const KP& p, const void* U, void* g, hipStream_t s) {
  return dispatch(p, U, g, s, true);
}

}  // namespace nedner

// Launch parameters shared by the host plan and the HIP kernels.
//
// One plain struct is passed by value to every kernel; it carries the sizes
// of the operator, the scalar constants of the window, frequency and weight
// (all reduced in double on the host) and the device tables of the plan.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.hpp"

namespace nedner {

enum Prec { PREC_FP64 = 0, PREC_FP32 = 1, PREC_FP32C = 2, PREC_FP32P = 3, PREC_FP32W = 4 };

struct KP {
  // ---- sizes -------------------------------------------------------------
  int M;          // sensors
  int Nt;         // time samples (even)
  int N1, N2, N3; // output voxels (even)
  int n1, n2;     // oversampled lateral grid sigma*N1, sigma*N2
  int ntt;        // time FFT length sigma*Nt
  int K2;         // half-spectrum columns along the second axis: N2/2 + 1
  int J1;         // first-axis columns kept: N1 + 1 (both Nyquist representatives)
  int W;          // window taps per dimension
  int TT;         // time samples per lane in spreading
  int S;          // mean rows per spreading sweep segment (the tuning parameter)
  int nseg;       // ceil(n1 / S)
  int CB;         // S + W
  int nsegt;      // sweep segments of all column groups (entries of segd)
  int nchunk;     // time chunks of 64*TT samples
  int prec;       // Prec
  int spread_pd;  // spreading sweep variant: 1 = samples staged through LDS (the only one)
  int wide_w;     // FP32W: 8-byte first-axis weights (fetched at use) instead of 4-byte
  int pass_lines; // FFT passes: lines per workgroup (power of two, upper bound)
  int pass_threads; // FFT passes: threads per workgroup (multiple of 64, <= 512)
  int pass_ip;    // FFT passes: in-place (1) or ping-pong (0) transform
  int window;     // 0: Gaussian exp(-beta x^2); 1: Kaiser-Bessel I0(beta sqrt(1 - (2x/W)^2))
  int equi;       // sensors on the output grid: placement instead of spreading, n1 = N1, n2 = N2
  int cosm;       // forward operator Q of the wave equation and its adjoint: the NER column
                  // values are averaged between l and -l (the cosine of the standing wave)
                  // and weighted by the constant scale_vol instead of W(j,l)

  // ---- window and frequency constants (double, reduced on the host) -----
  double beta;      // window parameter (see window), x in grid units, all three axes
  double cdtnt;     // c * dt * ntt: x(j,l) = sign(l) cdtnt |K|/(2 pi)
  double inv_L1sq;  // 1 / L1^2
  double inv_L2sq;  // 1 / L2^2
  double bz;        // 1 / (N3 d3)^2
  double phase_p;   // (Nt/2 + t0/dt) / ntt: phase/(2 pi) = x * phase_p
  double two_c;     // 2c
  double scale_vol; // (dt/d3) / (N1 N2 N3)
  double scale_spec;// dt/d3

  // ---- device tables (types follow the precision) ------------------------
  const void* w1;      // [M][W] weight type: s_m phi(o - f1), o = k - W/2 + 1
  const void* w2;      // [M][W] weight type: phi(o - f2)
  const int* cell;     // [M][2] (c1, c2)
  const int* ent_m;    // spreading list: sensor of each entry
  const void* ent_w2;  // spreading list: second-axis weight of each entry
  const int* cellbeg;  // list offsets per sweep cell: per segment, the tables of the four
                       // columns of its group, each S1 - S0 + W entries (cells Vstart..Vend, end)
  const int* segd;     // [nsegt][4] sweep segments: column group, S0, S1, offset of the first
                       // column's table in cellbeg (segments of a group consecutive)
  const int* node;     // equispaced: [n1 * n2] sensor at each node, -1 where none
  const int* gorder;   // [M] the sensors in the order the adjoint gather takes them: by tiles
                       // of 4 x 4 grid cells, so that consecutive sensors are neighbours
  const int* gcolbeg;  // [n2][n1 + 1] sweep gather: start of cell (c1, c2) in gcolm, per
                       // second-axis cell c2, c1 = 0..n1 (c1 = n1: end of the column)
  const int* gcolm;    // [M] sweep gather: the sensors by (c2, c1), index order within a cell
  int gS;              // sweep gather: first-axis cell rows per sweep segment (0: no sweep tables)
  const void* sw;      // equispaced: [M] real: h_m / (d1 d2)
  const void* dec1;    // [J1] real: 1/phihat_1(j1), j1 = -N1/2..N1/2
  const void* dec2;    // [K2] real: 1/phihat_2(k2), k2 = 0..N2/2
  const void* dect;    // [Nt] real: 1/phihat_t(n - Nt/2)
  const void* tw_n1;   // twiddles exp(-2 pi i k/n), complex of the data type
  const void* tw_n2;
  const void* tw_ntt;
  const void* tw_N1;
  const void* tw_N2;
  const void* tw_N3;
  Radices r_n1, r_n2, r_ntt, r_N1, r_N2, r_N3;
};

// The per-column transform buffer of the NER kernel holds max(ntt, N3)
// points plus COL_EXT periodic copies of its first points, so that a tap
// window never wraps (W <= COL_EXT).
constexpr int COL_EXT = 16;

// Workspace buffers of one execute (device pointers).
struct Bufs {
  void* U;   // spread grid        [n1][n2][Nt] real
  void* V;   // first FFT pass     [n1][K2][Nt] complex
  void* G;   // NED result columns [K2][J1][Nt] complex
  void* Z1;  // after depth IFFT   [K2][J1][N3] complex
  void* Z2;  // after first-axis IFFT [K2][N1][N3] complex
};

// Lines per workgroup of a batched FFT pass over lines of length n: the
// plan's upper bound, reduced to fit 160 KB of LDS and, in place, 8 points
// per thread. Shared by the single and the batched launches.
__host__ __device__ inline int pass_lines_for(const KP& p, int n, int cs) {
  int tb = p.pass_lines;
  while (tb > 1 && (long)n * cs * ((p.pass_ip ? 1 : 2) * (long)tb + 1) > 160 * 1024) tb >>= 1;
  while (p.pass_ip && tb > 1 && (long)n * tb > 8L * p.pass_threads) tb >>= 1;
  return tb;
}

// Allow a kernel more than 64 KB of dynamic LDS (gfx950 has 160 KB per CU).
template <typename F>
inline hipError_t allow_smem(F kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Host launchers (defined in the .hip files). All enqueue on `s` and return
// the launch status.
hipError_t launch_spread(const KP& p, const void* g, void* U, hipStream_t s);
// Equispaced sensors: U at each node = s_m g[m] (zero where no sensor), and its transpose.
hipError_t launch_place(const KP& p, const void* g, void* U, hipStream_t s);
hipError_t launch_place_adj(const KP& p, const void* U, void* g, hipStream_t s);
// Workgroups of the forward spreading kernel (prec, W, TT, wide_w of p) per CU.
int spread_blocks_per_cu(const KP& p);

// Image measures and projections (k_metrics.hip); the reductions use a
// caller workspace of METRICS_WORK_BYTES.
constexpr size_t METRICS_WORK_BYTES = 16384;
hipError_t launch_mip(const void* vol, int n1, int n2, int n3, int axis, bool dbl, void* out, hipStream_t s);
hipError_t launch_corrcoef(const void* a, const void* b, const unsigned char* mask, long n, bool dbl,
                           double* result, void* work, hipStream_t s);
hipError_t launch_tenenbaum(const void* img, long rows, long cols, long r0, long r1, long c0, long c1, bool dbl,
                            double scale, double* result, void* work, hipStream_t s);
// The correlation coefficient with its partial sums in a file-scope device
// array (k_metrics.hip) instead of a caller workspace: allocates nothing.
hipError_t launch_corrcoef_noalloc(const void* a, const void* b, const unsigned char* mask, long n, bool dbl,
                                   double* result, hipStream_t s);
size_t noalloc_scratch_bytes();
hipError_t launch_gather(const KP& p, const void* U, void* g, hipStream_t s);
hipError_t launch_lat_a(const KP& p, const void* U, void* V, hipStream_t s);
hipError_t launch_lat_b(const KP& p, const void* V, void* G, hipStream_t s);
hipError_t launch_column(const KP& p, const void* G, void* out, int spectrum, hipStream_t s);
hipError_t launch_pass_c(const KP& p, const void* Z1, void* Z2, hipStream_t s);
hipError_t launch_pass_d(const KP& p, const void* Z2, void* vol, hipStream_t s);
hipError_t launch_adj_d(const KP& p, const void* vol, void* Z2, hipStream_t s);
hipError_t launch_adj_c(const KP& p, const void* Z2, void* Z1, hipStream_t s);
hipError_t launch_column_adj(const KP& p, const void* Z1, void* G, hipStream_t s);
hipError_t launch_adj_b(const KP& p, const void* G, void* V, hipStream_t s);
hipError_t launch_adj_a(const KP& p, const void* V, void* U, hipStream_t s);

}  // namespace nedner

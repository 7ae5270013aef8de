// Image quality measures of App. B and maximum intensity projections.
//
//   corrcoef : Cov(a, b) / sqrt(Var(a) Var(b)) over the (masked) elements
//              (eq. (11)), in two passes: the means, then the centred second
//              moments, so that a large mean does not cancel the covariance;
//   tenenbaum: sum over the pixels of a rectangle whose 3x3 neighbourhood lies
//              in the image of (g * U)^2 + (g^T * U)^2, g the Sobel kernel
//              (eqs. (12)-(13)), optionally divided by the rectangle's element
//              count (the normalised measure App. B reports);
//   mip      : maximum along one axis of an (N1, N2, N3) volume, depth fastest.
//
// The sums accumulate in double. Every reduction runs on a fixed grid of
// MET_BLOCKS workgroups with a fixed-order tree in each and a fixed-order
// tree over the workgroups' partial sums, so repeated calls give identical
// results.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "kparams.hpp"

namespace nedner {

constexpr int MET_BLOCKS = 512;
constexpr int MET_THREADS = 256;

// Workspace (doubles): partial sums [3][MET_BLOCKS], then the means (2).
static_assert(sizeof(double) * (3 * MET_BLOCKS + 2) <= METRICS_WORK_BYTES, "metrics workspace");

// Sum NV values over the workgroup in a fixed order; the totals end in
// sh[k * MET_THREADS].
template <int NV>
__device__ __forceinline__ void block_sum(const double (&v)[NV], double* sh) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int k = 0; k < NV; ++k) sh[k * MET_THREADS + tid] = v[k];
  __syncthreads();
  for (int s = MET_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) {
#pragma unroll
      for (int k = 0; k < NV; ++k) sh[k * MET_THREADS + tid] += sh[k * MET_THREADS + tid + s];
    }
    __syncthreads();
  }
}

// PASS 0: sums of a, b and the count; PASS 1: centred products about the
// means left in the workspace by the PASS 0 finish.
template <typename T, int PASS>
__global__ __launch_bounds__(MET_THREADS) void k_moments(const T* __restrict__ a, const T* __restrict__ b,
                                                         const unsigned char* __restrict__ mask, long n,
                                                         double* __restrict__ work) {
  __shared__ double sh[3 * MET_THREADS];
  double v[3] = {0.0, 0.0, 0.0};
  double ma = 0.0, mb = 0.0;
  if (PASS == 1) {
    ma = work[3 * MET_BLOCKS];
    mb = work[3 * MET_BLOCKS + 1];
  }
  const long stride = (long)gridDim.x * MET_THREADS;
  for (long i = (long)blockIdx.x * MET_THREADS + threadIdx.x; i < n; i += stride) {
    if (mask && !mask[i]) continue;
    const double x = double(a[i]), y = double(b[i]);
    if (PASS == 0) {
      v[0] += x;
      v[1] += y;
      v[2] += 1.0;
    } else {
      const double dx = x - ma, dy = y - mb;
      v[0] += dx * dy;
      v[1] += dx * dx;
      v[2] += dy * dy;
    }
  }
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) work[k * MET_BLOCKS + blockIdx.x] = sh[k * MET_THREADS];
  }
}

// One workgroup: the three partial-sum rows, in a fixed tree. PASS 0 leaves
// the means in the workspace; PASS 1 writes the coefficient.
template <int PASS>
__global__ __launch_bounds__(MET_THREADS) void k_moments_finish(double* __restrict__ work,
                                                                double* __restrict__ result) {
  __shared__ double sh[3 * MET_THREADS];
  double v[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double t = 0.0;
    for (int j = threadIdx.x; j < MET_BLOCKS; j += MET_THREADS) t += work[k * MET_BLOCKS + j];
    v[k] = t;
  }
  block_sum<3>(v, sh);
  if (threadIdx.x == 0) {
    if (PASS == 0) {
      const double cnt = sh[2 * MET_THREADS];
      work[3 * MET_BLOCKS] = sh[0] / cnt;
      work[3 * MET_BLOCKS + 1] = sh[MET_THREADS] / cnt;
    } else {
      *result = sh[0] / sqrt(sh[MET_THREADS] * sh[2 * MET_THREADS]);
    }
  }
}

// Sobel responses at the pixels of [r0, r1) x [c0, c1) (already clamped to
// pixels with a full 3x3 neighbourhood), row-major image with `cols` columns.
template <typename T>
__global__ __launch_bounds__(MET_THREADS) void k_tenenbaum(const T* __restrict__ u, long cols, long r0, long r1,
                                                           long c0, long c1, double* __restrict__ work) {
  __shared__ double sh[MET_THREADS];
  double v[1] = {0.0};
  const long w = c1 - c0;
  const long total = (r1 > r0 && c1 > c0) ? (r1 - r0) * w : 0;
  const long stride = (long)gridDim.x * MET_THREADS;
  for (long i = (long)blockIdx.x * MET_THREADS + threadIdx.x; i < total; i += stride) {
    const long r = r0 + i / w, c = c0 + i % w;
    const T* up = u + (r - 1) * cols + c;
    const T* um = u + r * cols + c;
    const T* dn = u + (r + 1) * cols + c;
    const double a00 = double(up[-1]), a01 = double(up[0]), a02 = double(up[1]);
    const double a10 = double(um[-1]), a12 = double(um[1]);
    const double a20 = double(dn[-1]), a21 = double(dn[0]), a22 = double(dn[1]);
    // g = [[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]] and its transpose
    const double gx = (a02 - a00) + 2.0 * (a12 - a10) + (a22 - a20);
    const double gy = (a20 - a00) + 2.0 * (a21 - a01) + (a22 - a02);
    v[0] += gx * gx + gy * gy;
  }
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) work[blockIdx.x] = sh[0];
}

// The sum of the workgroups' partial sums times `scale` (1, or 1/N for the
// normalised measure).
__global__ __launch_bounds__(MET_THREADS) void k_sum_finish(const double* __restrict__ work, double scale,
                                                            double* __restrict__ result) {
  __shared__ double sh[MET_THREADS];
  double v[1] = {0.0};
  for (int j = threadIdx.x; j < MET_BLOCKS; j += MET_THREADS) v[0] += work[j];
  block_sum<1>(v, sh);
  if (threadIdx.x == 0) *result = sh[0] * scale;
}

// Maximum over the first (axis 0) or second (axis 1) index: one thread per
// output (a, i3), reading along the projected axis with stride `step`,
// coalesced along depth.
template <typename T>
__global__ __launch_bounds__(256) void k_mip_outer(const T* __restrict__ v, int n_axis, long step, int na,
                                                   long a_stride, int n3, T* __restrict__ out) {
  const long o = (long)blockIdx.x * 256 + threadIdx.x;
  if (o >= (long)na * n3) return;
  const long a = o / n3, i3 = o - a * n3;
  const T* p = v + a * a_stride + i3;
  T m = p[0];
  for (int k = 1; k < n_axis; ++k) m = fmax(m, p[k * step]);
  out[o] = m;
}

// Maximum over depth: one wavefront per (i1, i2) column, lanes striding the
// column, then a butterfly over the wavefront.
template <typename T>
__global__ __launch_bounds__(256) void k_mip_depth(const T* __restrict__ v, long ncol, int n3, T* __restrict__ out) {
  const long col = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (col >= ncol) return;
  const T* p = v + col * n3;
  T m = p[lane < n3 ? lane : 0];
  for (int i = lane + 64; i < n3; i += 64) m = fmax(m, p[i]);
#pragma unroll
  for (int s = 32; s > 0; s >>= 1) m = fmax(m, __shfl_xor(m, s, 64));
  if (lane == 0) out[col] = m;
}

template <typename T>
static hipError_t mip_t(const void* vol, int n1, int n2, int n3, int axis, void* out, hipStream_t s) {
  const T* v = static_cast<const T*>(vol);
  T* o = static_cast<T*>(out);
  if (axis == 2) {
    const long ncol = (long)n1 * n2;
    hipLaunchKernelGGL(k_mip_depth<T>, dim3(unsigned((ncol + 3) / 4)), dim3(256), 0, s, v, ncol, n3, o);
  } else {
    // axis 0: outputs (i2, i3), step n2 n3, a stride n3; axis 1: outputs
    // (i1, i3), step n3, a stride n2 n3
    const int na = axis == 0 ? n2 : n1;
    const int n_axis = axis == 0 ? n1 : n2;
    const long step = axis == 0 ? (long)n2 * n3 : (long)n3;
    const long a_stride = axis == 0 ? (long)n3 : (long)n2 * n3;
    const long total = (long)na * n3;
    hipLaunchKernelGGL(k_mip_outer<T>, dim3(unsigned((total + 255) / 256)), dim3(256), 0, s, v, n_axis, step, na,
                       a_stride, n3, o);
  }
  return hipGetLastError();
}

hipError_t launch_mip(const void* vol, int n1, int n2, int n3, int axis, bool dbl, void* out, hipStream_t s) {
  return dbl ? mip_t<double>(vol, n1, n2, n3, axis, out, s) : mip_t<float>(vol, n1, n2, n3, axis, out, s);
}

template <typename T>
static hipError_t corrcoef_t(const void* a, const void* b, const unsigned char* mask, long n, double* result,
                             void* work, hipStream_t s) {
  double* w = static_cast<double*>(work);
  const T* x = static_cast<const T*>(a);
  const T* y = static_cast<const T*>(b);
  hipLaunchKernelGGL((k_moments<T, 0>), dim3(MET_BLOCKS), dim3(MET_THREADS), 0, s, x, y, mask, n, w);
  hipLaunchKernelGGL(k_moments_finish<0>, dim3(1), dim3(MET_THREADS), 0, s, w, result);
  hipLaunchKernelGGL((k_moments<T, 1>), dim3(MET_BLOCKS), dim3(MET_THREADS), 0, s, x, y, mask, n, w);
  hipLaunchKernelGGL(k_moments_finish<1>, dim3(1), dim3(MET_THREADS), 0, s, w, result);
  return hipGetLastError();
}

hipError_t launch_corrcoef(const void* a, const void* b, const unsigned char* mask, long n, bool dbl,
                           double* result, void* work, hipStream_t s) {
  return dbl ? corrcoef_t<double>(a, b, mask, n, result, work, s)
             : corrcoef_t<float>(a, b, mask, n, result, work, s);
}

// ---------------------------------------------------------------- no allocation

// Scratch of the allocation-free correlation coefficient: the partial sums of
// the two passes and the means, in a file-scope device array instead of a
// caller workspace. Every device holds its own copy at its own address; host
// code reaches it only through the address hipGetSymbolAddress returns, taken
// once per device with that device current (the array's name in host code is
// a host-side stand-in, not a device address). Calls that overlap on one
// device share it and race.
constexpr int NOALLOC_SCRATCH_DOUBLES = 3 * MET_BLOCKS + 2;
static_assert(sizeof(double) * NOALLOC_SCRATCH_DOUBLES <= METRICS_WORK_BYTES, "no-allocation scratch");
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t noalloc_scratch_bytes() { return sizeof(double) * NOALLOC_SCRATCH_DOUBLES; }

// The current device's scratch address, looked up on the first call on that
// device (the device is current during the lookup).
hipError_t noalloc_scratch(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_corrcoef_noalloc(const void* a, const void* b, const unsigned char* mask, long n, bool dbl,
                                   double* result, hipStream_t s) {
  void* work = nullptr;
  const hipError_t e = noalloc_scratch(&work);
  if (e != hipSuccess) return e;
  // the kernels write every partial sum they read: nothing needs clearing
  return launch_corrcoef(a, b, mask, n, dbl, result, work, s);
}

hipError_t launch_tenenbaum(const void* img, long rows, long cols, long r0, long r1, long c0, long c1, bool dbl,
                            double scale, double* result, void* work, hipStream_t s) {
  r0 = r0 > 1 ? r0 : 1;
  c0 = c0 > 1 ? c0 : 1;
  r1 = r1 < rows - 1 ? r1 : rows - 1;
  c1 = c1 < cols - 1 ? c1 : cols - 1;
  double* w = static_cast<double*>(work);
  if (dbl)
    hipLaunchKernelGGL(k_tenenbaum<double>, dim3(MET_BLOCKS), dim3(MET_THREADS), 0, s,
                       static_cast<const double*>(img), cols, r0, r1, c0, c1, w);
  else
    hipLaunchKernelGGL(k_tenenbaum<float>, dim3(MET_BLOCKS), dim3(MET_THREADS), 0, s,
                       static_cast<const float*>(img), cols, r0, r1, c0, c1, w);
  hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(MET_THREADS), 0, s, w, scale, result);
  return hipGetLastError();
}

}  // namespace nedner

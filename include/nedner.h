/*
 * nedner.h - C-ABI of the NEDNER-NUFFT planar photoacoustic reconstruction
 * library for AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the discretised exact inversion formula for sensors
 * on a plane (Schmid et al., arXiv 1501.02946, eq. (1) and its non-equispaced
 * discretisation eq. (5), Sec. 2) with the three-step NEDNER-NUFFT of Sec. 3:
 *
 *   1. NED: a 2D non-uniform FFT over the sensor positions (eq. (9)-(10)):
 *      Gaussian spreading of every time sample onto an oversampled lateral
 *      grid, a lateral FFT and deconvolution;
 *   2. NER: a 1D non-uniform FFT in time evaluated at the frequencies
 *      omega = c sign(kz) |K| (eq. (6)-(8)), followed by the weight of eq. (1);
 *   3. an inverse 3D FFT to the image (Sec. 3, last step).
 *
 * and the exact transpose of that pipeline (the adjoint).
 *
 * Conventions (all physical units):
 *   sensor m at y_m = (y1, y2) on the plane z = 0 with detector area h_m,
 *   data g[m][n] recorded at t_n = t0 + n*dt, n = 0..nt-1, sound speed c;
 *   output voxel (i1, i2, i3) at (a1 + i1*d1, a2 + i2*d2, i3*d3); the lateral
 *   aperture [a_i, a_i + n_i*d_i) is periodic; d3 = 0 selects c*nt*dt/n3.
 *   Modes j_i in {-n_i/2..n_i/2-1}, k_i = 2 pi j_i/(n_i d_i),
 *   l in {-n3/2..n3/2-1}, kz = 2 pi l/(n3 d3), omega = c sign(l) |K|;
 *   W = 2c|kz|/|K| (l != 0), W(0,0) = 2c, W(j != 0, 0) = 0;
 *   F(j,l) = (dt/d3) W sum_n exp(-i omega t_n) sum_m h_m/(d1 d2) g[m][n] exp(-i k.(y_m - a));
 *   volume f = Re IDFT_3(F) / (n1 n2 n3).
 *
 * Layouts (row-major, last index fastest):
 *   data g      : [m][nt]            (FP64 plans: double, otherwise float)
 *   volume      : [n1][n2][n3]       real, depth fastest
 *   spectrum    : [n1][n2][n3]       complex (re, im interleaved), FFT order:
 *                                    index k along an axis holds mode k mod n
 *   stage grid  : [sigma*n1][sigma*n2][nt] real, the spread grid (debug)
 *
 * Ownership: plan creation copies every host array, so the caller may free
 * them on return. The plan owns its small device tables and frees them in
 * nedner_destroy. Large intermediates live in a caller-provided device
 * workspace (nedner_set_workspace) that must outlive every enqueued execute
 * and must not be shared by two executes in flight. Device pointers passed to
 * execute calls belong to the caller and must be on the plan's device.
 * Execute calls are asynchronous on the given HIP stream (NULL = default).
 *
 * Errors: no call aborts or throws across this interface. Each returns a
 * status; nedner_last_error() gives a thread-local message for the last
 * failing call on that thread. After NEDNER_E_HIP a plan accepts only
 * nedner_destroy. Plans are independent; one plan is not reentrant.
 */
#ifndef NEDNER_H
#define NEDNER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NEDNER_VERSION 100

typedef struct nedner_plan_s* nedner_plan;

typedef enum {
  NEDNER_OK = 0,
  NEDNER_E_ARG = 1,          /* invalid descriptor or argument */
  NEDNER_E_ALIAS = 2,        /* max |omega| dt >= pi and ALLOW_ALIAS not set */
  NEDNER_E_OOM = 3,          /* device or host allocation failed */
  NEDNER_E_WORKSPACE = 4,    /* no workspace, or one that is too small */
  NEDNER_E_HIP = 5,          /* a HIP runtime call failed; plan is now unusable */
  NEDNER_E_UNSUPPORTED = 6,  /* valid but not implemented (FFT size, kind) */
  NEDNER_E_STATE = 7         /* plan unusable after an earlier HIP error */
} nedner_status;

/* Arithmetic of a plan. "Arguments" are the window and phase arguments:
   the grid coordinates of the sensors (plan time, host), x(j,l) = omega dt
   ntt/(2 pi) and the phase (N_t/2 theta + omega t0) mod 2 pi (NER kernels). */
typedef enum {
  NEDNER_FP64 = 0,              /* every step in double */
  NEDNER_FP32 = 1,              /* float data, sums and transforms; double arguments */
  NEDNER_FP32_COMPENSATED = 2,  /* as FP32, with compensated float sums where many terms meet:
                                   the spreading holds each grid value as a pair hi + lo of
                                   floats, adds terms to lo and folds lo into hi with Kahan's
                                   update after every 16 terms (blocked compensated summation),
                                   rounding hi + lo once; the adjoint gather adds its W row
                                   sums with Kahan's update */
  NEDNER_FP32_PLAIN = 3,        /* float everywhere, arguments included */
  NEDNER_FP32_WIDE = 4          /* float data; spreading sums, the adjoint gather's row-sum
                                   merges and the first-axis spreading weights in double */
} nedner_precision;

/* Element type of the image measures' inputs. */
typedef enum {
  NEDNER_DTYPE_F32 = 0,
  NEDNER_DTYPE_F64 = 1
} nedner_dtype;

/* Interpolation window of the spreading (eq. (10)) and of the NER gather
   (eq. (8)), the same on all three axes, W taps per axis around each point.
   Gaussian: phi(x) = exp(-beta x^2), beta = pi (sigma - 1/2) / (sigma W/2) / tau_scale
     (Greengard and Lee, SIAM Rev. 46 (2004)), phihat(xi) = sqrt(pi/beta) exp(-pi^2 xi^2/beta).
   Kaiser-Bessel (the paper's window, Sec. 3): phi(x) = I0(beta sqrt(1 - (2x/W)^2)) for
     |x| < W/2, beta = pi sqrt((W/sigma)^2 (sigma - 1/2)^2 - 0.8) (Beatty, Nishimura and
     Pauly, IEEE TMI 24 (2005)), phihat(xi) = W sinh(z)/z with z = sqrt(beta^2 - (pi W xi)^2)
     (sin(|z|)/|z| past the cut-off). It reaches a given accuracy with fewer taps;
     it is built for w = 4..12 (NEDNER_E_UNSUPPORTED otherwise).
   x is in oversampled grid units, xi in cycles per grid unit. */
typedef enum {
  NEDNER_WINDOW_GAUSSIAN = 0,
  NEDNER_WINDOW_KAISER_BESSEL = 1
} nedner_window;

typedef enum {
  NEDNER_VOLUME_REAL = 0,       /* the image f, [n1][n2][n3] real */
  NEDNER_SPECTRUM_COMPLEX = 1,  /* F(j,l), [n1][n2][n3] complex, FFT order */
  NEDNER_STAGE_GRID = 2         /* the spread grid (forward) / its transpose (adjoint) */
} nedner_kind;

#define NEDNER_ALLOW_ALIAS 1u      /* accept max |omega| dt >= pi */
#define NEDNER_WRAP_POSITIONS 2u   /* wrap positions into the periodic aperture */
#define NEDNER_DETERMINISTIC 4u    /* accepted; every path is bitwise deterministic */
#define NEDNER_NO_AUTOTUNE 8u      /* keep the built-in launch shapes */
/* Sensors on the output grid (the NER-NUFFT case, Sec. 3 eq. (4)): every
   position is a voxel node a + i d (i integer in [0, n)), at most one sensor
   per node. The lateral sums of eq. (5) are then a plain DFT of the
   zero-filled node grid: no spreading, no lateral window or oversampling,
   only the time axis keeps the window. Positions off the grid are
   NEDNER_E_ARG; batched plans reject the flag (NEDNER_E_UNSUPPORTED). */
#define NEDNER_EQUISPACED 16u

/* Plan descriptor. Fill with nedner_desc_init, then set the fields. */
typedef struct {
  int64_t m;            /* number of sensors, >= 1 */
  const double* xy;     /* host, [m][2] positions (y1, y2) */
  const double* h;      /* host, [m] detector areas; NULL => n1 d1 n2 d2 / m each */
  int64_t nt;           /* time samples, even, >= 2 */
  double t0, dt, c;     /* first sample time, time step > 0, sound speed > 0 */
  int32_t n1, n2, n3;   /* output voxels, each even and >= 2; n2 = 1 is the two-dimensional
                           problem (sensors on a line along the first axis, image (i1, i3),
                           the second axis carrying only the mode k2 = 0; not with
                           NEDNER_EQUISPACED) */
  double a1, a2;        /* aperture origin */
  double d1, d2, d3;    /* voxel steps; d1, d2 > 0; d3 = 0 => c nt dt / n3 */
  int32_t prec;         /* nedner_precision */
  int32_t w;            /* window taps per dimension, even, 2..16 (default 12 = 2K, K = 6) */
  double sigma;         /* oversampling factor (default 2); sigma*n1, sigma*n2,
                           sigma*nt must be even integers */
  double tau_scale;     /* Gaussian width scale relative to Greengard-Lee (default 1) */
  uint32_t flags;       /* NEDNER_* flags */
  int32_t rows_per_wave;   /* spreading sweep length; 0 = automatic */
  int32_t time_per_lane;   /* time samples per lane in spreading (1, 2, 4); 0 = automatic */
  int32_t window;          /* nedner_window (default Gaussian); tau_scale applies to the Gaussian */
} nedner_desc;

/* Sizes a descriptor implies; filled by nedner_query (host only, no HIP). */
typedef struct {
  int32_t n1_os, n2_os, nt_os;   /* oversampled lateral grid and time FFT length */
  int32_t columns;               /* NER columns: (n1 + 1) * (n2 / 2 + 1) */
  int32_t segments;              /* spreading sweep segments along the first axis */
  int32_t rows_per_wave;         /* rows per sweep segment */
  int32_t time_per_lane;         /* time samples per lane in spreading */
  int32_t pad0;
  size_t workspace_bytes;        /* device workspace an execute needs */
  size_t table_bytes;            /* device tables the plan allocates */
  double beta;                   /* window parameter beta (see nedner_window) */
  double max_abs_theta;          /* max |omega| dt over the mode set (alias check: < pi) */
  int64_t list_entries;          /* (sensor, column) pairs in the spreading lists */
} nedner_info;

/* Launch shape of a plan: what the autotuner chooses. Accuracy parameters
   (w, sigma, tau_scale) are never part of it. */
typedef struct {
  int32_t rows_per_wave;   /* spreading sweep length (rows of the oversampled grid) */
  int32_t time_per_lane;   /* spreading time samples per lane: 1, 2 or 4 */
  int32_t spread_depth;    /* spreading sweep variant: 1 = samples staged through LDS in
                              batches (the only one; other values are NEDNER_E_ARG) */
  int32_t pass_lines;      /* FFT passes: lines per workgroup (power of two) */
  int32_t pass_threads;    /* FFT passes: threads per workgroup (64..512, multiple of 64) */
  int32_t pass_inplace;    /* FFT passes: in-place (1) or ping-pong (0) transform */
  int32_t gather_rows;     /* adjoint gather: first-axis cell rows per sweep segment of the
                              sweep gather (float plans, w <= 12), or 0: the tile-staged
                              gather (the only one of FP64 plans and w > 12) */
  int32_t pad1;
  double ms_spread;        /* autotune: spreading time of the chosen shape, ms */
  double ms_execute;       /* autotune: forward execute time of the chosen shape, ms */
} nedner_tuning;

/* Fill a descriptor with the defaults (w = 12, sigma = 2, tau_scale = 1, FP32,
   Gaussian window). */
void nedner_desc_init(nedner_desc* desc);

/* Host-only validation of a descriptor (no HIP call): the sizes, steps and
   flags of the problem statement of Sec. 2 (sensors on the plane, samples at
   t0 + n dt, voxels a + i d) and the aliasing bound max |omega| dt < pi of the
   time sampling (eq. (1) evaluated at the frequencies of eq. (5)). Returns
   NEDNER_E_ARG, NEDNER_E_ALIAS, NEDNER_E_UNSUPPORTED or NEDNER_OK. */
nedner_status nedner_validate(const nedner_desc* desc);

/* Host-only: validate and report in *info the sizes the plan would use
   (oversampled grid, list entries, workspace bytes). No HIP call. */
nedner_status nedner_query(const nedner_desc* desc, nedner_info* info);

/* Build a plan on `device` for the operator of eq. (5) (Sec. 2) evaluated by
   the NEDNER-NUFFT of Sec. 3: every sensor's grid coordinate is split into a
   cell and a fraction in FP64 and its window weights are tabulated (the
   "nearest integers" of the NED step, eq. (10)); the per-column spreading
   lists, the deconvolution tables 1/phihat of eqs. (8) and (10) and the
   twiddle tables are built and uploaded. `desc` and its host arrays xy
   ([m][2] double) and h ([m] double or NULL) are read during the call only.
   `stream` is accepted for symmetry and not used (uploads are synchronous).
   On success *plan owns the device tables until nedner_destroy; the
   workspace is still to be set. Errors: the statuses of nedner_validate,
   NEDNER_E_OOM (host or device allocation), NEDNER_E_HIP (device selection
   or upload); *plan is left untouched on failure. */
nedner_status nedner_plan_create(const nedner_desc* desc, int device, void* stream,
                                 nedner_plan* plan);

/* Batched plan: `count` independent problems (descs[0..count-1], one
   precision, window and window width; sizes and sensors may differ) run
   together by the *_many calls, one persistent launch per pipeline stage.
   Errors as nedner_plan_create, NEDNER_E_ARG for mixed precision or window. */
nedner_status nedner_plan_create_many(const nedner_desc* descs, int count, int device,
                                      void* stream, nedner_plan* plan);

nedner_status nedner_plan_info(nedner_plan plan, nedner_info* info);
nedner_status nedner_workspace_size(nedner_plan plan, size_t* bytes);
/* Attach a device workspace of at least nedner_workspace_size bytes (256-byte
   aligned), owned by the caller, on the plan's device. It must outlive every
   enqueued execute and must not serve two executes in flight. NULL detaches.
   NEDNER_E_WORKSPACE when smaller than needed, NEDNER_E_ARG when misaligned. */
nedner_status nedner_set_workspace(nedner_plan plan, void* d_workspace, size_t bytes);

/* The reconstruction of Sec. 3: eq. (5) evaluated by the NED step (spreading
   of eq. (10), lateral FFT, deconvolution), the NER step (time FFT and the
   interpolation of eq. (8) at omega = c sign(kz)|K|, with the weight of
   eq. (1)) and the closing inverse 3D FFT. d_g: device [m][nt] data of the
   plan's type (double for NEDNER_FP64, float otherwise), time fastest.
   d_out: device output of `kind`: NEDNER_VOLUME_REAL [n1][n2][n3] real,
   NEDNER_SPECTRUM_COMPLEX [n1][n2][n3] complex in FFT order (no closing
   inverse FFT), NEDNER_STAGE_GRID the spread grid [sigma n1][sigma n2][nt]
   (no workspace needed). Both buffers belong to the caller; d_out is written
   completely. Asynchronous on `stream` (a HIP stream of the plan's device,
   NULL = default). Errors (nothing is launched): NEDNER_E_ARG (NULL plan or
   pointer, unknown kind, batched plan), NEDNER_E_WORKSPACE (no workspace or
   too small), NEDNER_E_STATE (after an earlier HIP error); NEDNER_E_HIP when a
   launch fails (the plan then accepts only nedner_destroy). */
nedner_status nedner_execute(nedner_plan plan, const void* d_g, void* d_out, int kind,
                             void* stream);

/* The exact transpose of nedner_execute for the real Euclidean inner
   products on data and volume (it is not in the paper; it makes the
   reconstruction usable as a differentiable operator): d_in of `kind`
   (NEDNER_VOLUME_REAL [n1][n2][n3] or NEDNER_STAGE_GRID, the transpose of the
   spreading alone) -> d_g [m][nt]. Types, ownership, stream and errors as for
   nedner_execute; NEDNER_SPECTRUM_COMPLEX is NEDNER_E_UNSUPPORTED. */
nedner_status nedner_execute_adjoint(nedner_plan plan, const void* d_in, int kind, void* d_g,
                                     void* stream);

/* Forward operator Q of the wave equation (Sec. 2): initial pressure -> the
   trace, at the sensors on the plane z = 0, of the solution of the wave
   equation with sound speed c, p(., 0) = v and zero initial velocity, for the
   volume taken as periodic on the voxel grid (period N_i d_i per axis):
     g[m][n] = Re sum_{j,l} V(j,l) cos(c |K(j,l)| t_n) exp(i k_j.(y_m - a)),
     V = DFT_3(v) / (N1 N2 N3),  t_n = t0 + n dt,
   with the same modes, wavenumbers and window approximations as the plan's
   reconstruction, no sensor weight h_m and no inversion weight. It runs the
   plan's adjoint pipeline with each NER column averaged between l and -l
   (cos(omega t) = (exp(i omega t) + exp(-i omega t))/2 and omega(-l) =
   -omega(l)). d_v: device (N1, N2, N3) of the plan's data type, depth
   fastest; d_g: device (m, nt) output. Needs the workspace; not for batched
   plans (NEDNER_E_ARG). Asynchronous on `stream`. */
nedner_status nedner_execute_q(nedner_plan plan, const void* d_v, void* d_g, void* stream);

/* Adjoint of nedner_execute_q for the real Euclidean inner products: data
   d_g (m, nt) -> volume d_v (N1, N2, N3),
     v = Re IDFT_3(C),  C(j,l) = sum_n G(j,n) cos(c |K(j,l)| t_n),
     G(j,n) = sum_m d_g[m][n] exp(-i k_j.(y_m - a)),
   the plan's forward pipeline with unit sensor weights, the constant weight
   1/(N1 N2 N3) and each column averaged between l and -l. Same buffers,
   workspace and errors as nedner_execute_q. */
nedner_status nedner_execute_q_adjoint(nedner_plan plan, const void* d_g, void* d_v, void* stream);

/* Testing hook for the error path: puts the plan into the state a failed
   HIP call leaves (as if a HIP call of the plan had returned `code`, which
   must not be hipSuccess) and returns NEDNER_E_HIP with that call's message
   in nedner_last_error. Launches nothing and touches no device memory.
   Afterwards every execute, tuning and profiling call on the plan returns
   NEDNER_E_STATE; nedner_destroy still releases it. NULL plan: NEDNER_E_ARG. */
nedner_status nedner_debug_inject_hip_error(nedner_plan plan, int code);

/* Batched forward (the reconstruction of nedner_execute for every problem
   of a plan_create_many plan, one persistent launch per stage over all of
   them): host arrays of `count` device pointers, d_g[i] the [m_i][nt_i] data
   and d_out[i] the [n1_i][n2_i][n3_i] volume of problem i. Only
   NEDNER_VOLUME_REAL. Each problem's result is bitwise equal to its own
   single-problem plan's. Errors as nedner_execute. */
nedner_status nedner_execute_many(nedner_plan plan, const void* const* d_g,
                                  void* const* d_out, int kind, void* stream);

/* Release a plan and its device tables (freed with hipFree, which waits for
   the device's pending work). The caller's workspace and buffers are not
   touched. NULL is accepted. */
nedner_status nedner_destroy(nedner_plan plan);

/* ---- image measures (App. B) and projections: no plan needed ----------- */

/* Device workspace (bytes) of nedner_corrcoef and nedner_tenenbaum. */
size_t nedner_metrics_workspace_size(void);

/* Maximum intensity projection of a device volume (n1, n2, n3), depth
   fastest, along `axis` (0, 1 or 2) into d_out: (n2, n3), (n1, n3) or
   (n1, n2), row-major, same dtype. Inputs are assumed finite. */
nedner_status nedner_mip(const void* d_vol, int n1, int n2, int n3, int axis, int dtype, void* d_out,
                         void* stream);

/* Correlation coefficient of two device arrays of n elements (App. B,
   eq. (11)): Cov(a, b) / sqrt(Var(a) Var(b)) over the elements whose mask
   byte is non-zero (all elements when d_mask is NULL), in two passes (means,
   then centred sums) accumulated in double. The result goes to the device
   double *d_result (NaN when a variance is zero or no element is selected).
   d_work: device workspace of nedner_metrics_workspace_size() bytes, not
   shared with a concurrent call. Deterministic. */
nedner_status nedner_corrcoef(const void* d_a, const void* d_b, const unsigned char* d_mask, int64_t n,
                              int dtype, double* d_result, void* d_work, size_t work_bytes, void* stream);

/* nedner_corrcoef for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same kernels and the same result, bit for bit, with the partial sums
   in a file-scope device array of 12 304 bytes (3 * 512 + 2 doubles) that
   every device the library runs on holds until the process ends, instead of
   a caller workspace. That size does not depend on n, so no input is too
   large for it. The array's device address is looked up once per device, on
   the first call made with that device current. Every call on a device
   shares its array: calls that overlap on one device (concurrent streams or
   threads) race and must be serialised by the caller. Allocates nothing
   (no hipMalloc, hipFree or allocating library call); the kernels write every
   scratch value they read, so nothing is cleared between calls. Arguments
   and errors as nedner_corrcoef without the workspace; NEDNER_E_HIP if the
   scratch address cannot be obtained. */
nedner_status nedner_corrcoef_noalloc(const void* d_a, const void* d_b, const unsigned char* d_mask, int64_t n,
                                      int dtype, double* d_result, void* stream);

/* Tenenbaum sharpness of a device image (rows, cols), row-major (App. B,
   eqs. (12)-(13)): the sum of (g * U)^2 + (g^T * U)^2, g the 3x3 Sobel kernel
   [[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]], over the pixels of the half-open
   rectangle [r0, r1) x [c0, c1) whose 3x3 neighbourhood lies inside the
   image; accumulated in double into *d_result. Same workspace rules as
   nedner_corrcoef. */
nedner_status nedner_tenenbaum(const void* d_img, int64_t rows, int64_t cols, int64_t r0, int64_t r1,
                               int64_t c0, int64_t c1, int dtype, double* d_result, void* d_work,
                               size_t work_bytes, void* stream);

/* The normalised Tenenbaum measure App. B reports (after eqs. (12)-(13)):
   the sum of nedner_tenenbaum divided by N, the number of elements of the
   image it is taken over, here the rectangle [r0, r1) x [c0, c1) as given
   (0 for an empty rectangle). Arguments, workspace and errors as for
   nedner_tenenbaum. */
nedner_status nedner_tenenbaum_mean(const void* d_img, int64_t rows, int64_t cols, int64_t r0, int64_t r1,
                                    int64_t c0, int64_t c1, int dtype, double* d_result, void* d_work,
                                    size_t work_bytes, void* stream);

/* Current launch shape of a plan (of its first problem for a batch). */
nedner_status nedner_get_tuning(nedner_plan plan, nedner_tuning* tuning);

/* Apply a launch shape (e.g. one cached from an earlier autotune) to a
   single-problem plan; rebuilds the spreading lists when the sweep changes.
   Synchronises the device. Returns NEDNER_E_ARG for an invalid shape. */
nedner_status nedner_set_tuning(nedner_plan plan, const nedner_tuning* tuning);

/* Measure candidate launch shapes with HIP events on `stream` and keep the
   fastest: sweep length and time samples per lane of the spreading (timed
   alone), the sweep segment of the adjoint gather (timed alone, on the
   spread grid), then the FFT pass shape (timed on a whole forward execute).
   `d_g` is one data array of the plan's problem (any values, never written;
   for a batch, NULL: the batch's spreading launch is timed on zero data in
   its workspace slices with the batch's samples per lane kept). Needs the
   workspace. Synchronises the device; allocates a temporary volume and
   data array. */
nedner_status nedner_autotune(nedner_plan plan, const void* d_g, void* stream, nedner_tuning* best);

/* Stage timing with HIP events recorded on the execute stream, for up to
   `max_runs` following executes (forward or adjoint). nedner_profile_end
   waits for them and writes the mean milliseconds of each stage into
   ms[0..*n_stages-1] (at most max_stages), in pipeline order; `names` (may be
   NULL) receives a static comma-separated list of the stage names. Profiling
   adds two event records per stage and no synchronisation. */
nedner_status nedner_profile_begin(nedner_plan plan, int max_runs);
nedner_status nedner_profile_end(nedner_plan plan, double* ms, int max_stages, int* n_stages,
                                 const char** names);

const char* nedner_status_string(nedner_status status);
const char* nedner_last_error(void);
int nedner_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NEDNER_H */

// C-ABI of the NEDNER library: validation, plan construction and execution.
//
// Plan construction does the host-side geometry in double: every sensor's
// grid coordinate u = n (y - a)/L is split into an integer cell and a
// fraction, the window weights phi(o - frac) are tabulated per sensor and axis
// (the "nearest integers" of eq. (10)), and the per-column spreading lists are
// built. Nothing of that depends on the data, so execute only runs kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "batch.hpp"
#include "nedner.h"

using nedner::KP;
using nedner::Radices;

namespace {

thread_local std::string g_last_error;

nedner_status fail(nedner_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

bool finite(double v) { return std::isfinite(v); }

bool five_smooth(long n) {
  if (n < 1) return false;
  for (long p : {2L, 3L, 5L})
    while (n % p == 0) n /= p;
  return n == 1;
}

// Integer value of sigma * n when it is one (within 1e-9), else -1.
long scaled_size(double sigma, long n) {
  const double v = sigma * double(n);
  const double r = std::floor(v + 0.5);
  if (std::fabs(v - r) > 1e-9 * std::max(1.0, v)) return -1;
  return long(r);
}

Radices make_radices(int n) {
  Radices rd{};
  rd.n = n;
  int m = n, c = 0;
  int e2 = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++e2;
  }
  while (e2 >= 3) {
    rd.r[c++] = 8;
    e2 -= 3;
  }
  if (e2 == 2) rd.r[c++] = 4;
  if (e2 == 1) rd.r[c++] = 2;
  while (m % 5 == 0) {
    m /= 5;
    rd.r[c++] = 5;
  }
  while (m % 3 == 0) {
    m /= 3;
    rd.r[c++] = 3;
  }
  rd.count = c;
  return rd;
}

struct Derived {
  long n1, n2, ntt;
  double L1, L2, D3, beta;
  int W, TT, S, nseg, nchunk, CB, K2, J1;
  int window;
  bool equi;  // sensors on the output grid: no lateral spreading or oversampling
  double max_theta;
};

// Modified Bessel function I0 by its power series sum_k (x^2/4)^k / (k!)^2,
// summed until a term no longer changes the (all positive) sum.
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 1000; ++k) {
    term *= q / (double(k) * double(k));
    const double next = sum + term;
    if (next == sum) break;
    sum = next;
  }
  return sum;
}

// The window and its Fourier transform (nedner_window), x and xi in grid units.
double window_phi(const Derived& v, double x) {
  if (v.window == NEDNER_WINDOW_KAISER_BESSEL) {
    const double a = 2.0 * x / v.W;
    return std::fabs(a) < 1.0 ? bessel_i0(v.beta * std::sqrt(1.0 - a * a)) : 0.0;
  }
  return std::exp(-v.beta * x * x);
}

// phihat at mode k of an n-point grid: xi = k / n
double window_phihat(const Derived& v, double k, double n) {
  const double xi = k / n;
  if (v.window == NEDNER_WINDOW_KAISER_BESSEL) {
    const double w = M_PI * v.W * xi;
    const double z2 = v.beta * v.beta - w * w;
    if (z2 > 0) {
      const double z = std::sqrt(z2);
      return v.W * std::sinh(z) / z;
    }
    if (z2 < 0) {
      const double z = std::sqrt(-z2);
      return v.W * std::sin(z) / z;
    }
    return double(v.W);
  }
  return std::sqrt(M_PI / v.beta) * std::exp(-M_PI * M_PI * xi * xi / v.beta);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t real_size(int prec) { return prec == NEDNER_FP64 ? 8 : 4; }
// Tuning override read at plan creation: NEDNER_SPREAD="1,wide" keeps the
// one spreading sweep (samples staged through LDS) and sets, for FP32W,
// 8-byte first-axis weights (wide = 1, the default) or 4-byte ones (0).
struct SpreadOpt {
  int pd = 1, wide = 1;
};
SpreadOpt spread_opt() {
  SpreadOpt o;
  if (const char* e = getenv("NEDNER_SPREAD")) {
    int a = 0, b = 0;
    if (sscanf(e, "%d,%d", &a, &b) == 2 && a == 1) o.wide = b != 0;
  }
  return o;
}

size_t weight_size(int prec) {
  return prec == NEDNER_FP64 || (prec == NEDNER_FP32_WIDE && spread_opt().wide) ? 8 : 4;
}

// Workspace: buffer 0 holds U, then G, then Z2; buffer 1 holds V, then Z1.
void workspace_layout(const nedner_desc& d, const Derived& v, size_t* off1, size_t* total) {
  const size_t rs = real_size(d.prec), cs = 2 * rs;
  const size_t U = (size_t)v.n1 * v.n2 * d.nt * rs;
  const size_t V = (size_t)v.n1 * v.K2 * d.nt * cs;
  const size_t G = (size_t)v.K2 * v.J1 * d.nt * cs;
  const size_t Z1 = (size_t)v.K2 * v.J1 * d.n3 * cs;
  const size_t Z2 = (size_t)v.K2 * d.n1 * d.n3 * cs;
  const size_t b0 = align256(std::max(U, std::max(G, Z2)));
  const size_t b1 = align256(std::max(V, Z1));
  *off1 = b0;
  *total = b0 + b1;
}

// LDS of a column workgroup with one column: shared twiddles + one wave's buffers.
size_t column_lds(const nedner_desc& d, const Derived& v) {
  const size_t rs = real_size(d.prec), cs = 2 * rs;
  const size_t nbuf = std::max<size_t>(v.ntt, d.n3) + nedner::COL_EXT;
  const size_t wave = (cs * (nbuf + d.n3 + 1) + (rs + 4) * (d.n3 + 1) + 15) & ~size_t(15);
  // half-period twiddle tables; the depth table shares the time table when n3 divides ntt
  return cs * (v.ntt / 2 + (v.ntt % d.n3 ? d.n3 / 2 : 0)) + wave;
}

// Node (i1, i2) of sensor m when it sits on the output grid a + i d (after
// wrapping into the aperture): |u - round(u)| <= 1e-9 with u = (y - a)/d.
bool grid_node(const nedner_desc& d, const Derived& v, int64_t m, long* i) {
  const double L[2] = {v.L1, v.L2}, a[2] = {d.a1, d.a2}, st[2] = {d.d1, d.d2};
  const long n[2] = {d.n1, d.n2};
  for (int ax = 0; ax < 2; ++ax) {
    double y = d.xy[2 * m + ax] - a[ax];
    y -= L[ax] * std::floor(y / L[ax]);
    const double u = y / st[ax];
    const double r = std::nearbyint(u);
    if (std::fabs(u - r) > 1e-9) return false;
    i[ax] = long(r) % n[ax];
  }
  return true;
}

nedner_status validate_impl(const nedner_desc* d, Derived* out) {
  if (!d) return fail(NEDNER_E_ARG, "descriptor is NULL");
  if (d->m < 1 || d->m > (int64_t(1) << 30)) return fail(NEDNER_E_ARG, "m must be in [1, 2^30]");
  if (!d->xy) return fail(NEDNER_E_ARG, "xy is NULL");
  if (d->nt < 2 || (d->nt % 2) || d->nt > (1 << 20)) return fail(NEDNER_E_ARG, "nt must be even and in [2, 2^20]");
  if (!finite(d->t0) || !finite(d->dt) || !(d->dt > 0)) return fail(NEDNER_E_ARG, "t0 must be finite and dt > 0");
  if (!finite(d->c) || !(d->c > 0)) return fail(NEDNER_E_ARG, "c must be finite and > 0");
  // n2 = 1 is the two-dimensional problem (d = 2 in Sec. 2): sensors on a line
  // along the first axis, one voxel across the second, image (i1, i3)
  auto even_size = [](int n) { return n >= 2 && n % 2 == 0 && n <= (1 << 16); };
  if (!even_size(d->n1) || !even_size(d->n3) || !(even_size(d->n2) || d->n2 == 1))
    return fail(NEDNER_E_ARG, "n1, n3 must be even and in [2, 65536]; n2 too, or 1 for the 2-D problem");
  if (!finite(d->a1) || !finite(d->a2)) return fail(NEDNER_E_ARG, "a1, a2 must be finite");
  if (!finite(d->d1) || !finite(d->d2) || !(d->d1 > 0) || !(d->d2 > 0))
    return fail(NEDNER_E_ARG, "d1, d2 must be finite and > 0");
  if (!finite(d->d3) || d->d3 < 0) return fail(NEDNER_E_ARG, "d3 must be finite and >= 0");
  if (d->prec < 0 || d->prec > 4) return fail(NEDNER_E_ARG, "unknown precision");
  if (d->w < 2 || d->w > 16 || (d->w % 2)) return fail(NEDNER_E_ARG, "w must be even and in [2, 16]");
  if (!finite(d->sigma) || !(d->sigma > 1.0)) return fail(NEDNER_E_ARG, "sigma must be finite and > 1");
  if (!finite(d->tau_scale) || !(d->tau_scale > 0)) return fail(NEDNER_E_ARG, "tau_scale must be finite and > 0");
  if (d->rows_per_wave < 0) return fail(NEDNER_E_ARG, "rows_per_wave must be >= 0");
  if (d->time_per_lane != 0 && d->time_per_lane != 1 && d->time_per_lane != 2 && d->time_per_lane != 4)
    return fail(NEDNER_E_ARG, "time_per_lane must be 0, 1, 2 or 4");
  if (d->flags & ~uint32_t(31)) return fail(NEDNER_E_ARG, "unknown flag bits");
  Derived v{};
  v.equi = (d->flags & NEDNER_EQUISPACED) != 0;
  v.n1 = v.equi ? d->n1 : scaled_size(d->sigma, d->n1);
  v.n2 = v.equi ? d->n2 : scaled_size(d->sigma, d->n2);
  v.ntt = scaled_size(d->sigma, d->nt);
  if (v.n1 < 0 || v.n2 < 0 || v.ntt < 0 || (v.n1 % 2) || (v.n2 % 2) || (v.ntt % 2))
    return fail(NEDNER_E_ARG, "sigma * n1, sigma * n2 and sigma * nt must be even integers");
  v.L1 = d->n1 * d->d1;
  v.L2 = d->n2 * d->d2;
  v.D3 = d->d3 > 0 ? d->d3 : d->c * double(d->nt) * d->dt / d->n3;
  v.W = d->w;
  if (d->window != NEDNER_WINDOW_GAUSSIAN && d->window != NEDNER_WINDOW_KAISER_BESSEL)
    return fail(NEDNER_E_ARG, "unknown window");
  v.window = d->window;
  if (v.window == NEDNER_WINDOW_KAISER_BESSEL && (d->w < 4 || d->w > 12))
    return fail(NEDNER_E_UNSUPPORTED, "the Kaiser-Bessel window is built for 4 to 12 taps");
  if (v.window == NEDNER_WINDOW_KAISER_BESSEL) {
    const double r = (d->w / d->sigma) * (d->sigma - 0.5);
    if (r * r <= 0.8) return fail(NEDNER_E_ARG, "Kaiser-Bessel window needs (w/sigma)^2 (sigma-1/2)^2 > 0.8");
    v.beta = M_PI * std::sqrt(r * r - 0.8);
  } else {
    v.beta = M_PI * (d->sigma - 0.5) / (d->sigma * (d->w / 2.0)) / d->tau_scale;
  }
  v.K2 = d->n2 / 2 + 1;
  v.J1 = d->n1 + 1;
  // positions
  const bool wrap = (d->flags & NEDNER_WRAP_POSITIONS) != 0;
  for (int64_t m = 0; m < d->m; ++m) {
    const double y1 = d->xy[2 * m], y2 = d->xy[2 * m + 1];
    if (!finite(y1) || !finite(y2)) return fail(NEDNER_E_ARG, "non-finite sensor position at index " + std::to_string(m));
    if (!wrap && (y1 < d->a1 || y1 >= d->a1 + v.L1 || y2 < d->a2 || y2 >= d->a2 + v.L2))
      return fail(NEDNER_E_ARG, "sensor " + std::to_string(m) + " outside the aperture (set NEDNER_WRAP_POSITIONS to wrap)");
    if (d->h) {
      const double h = d->h[m];
      if (!finite(h) || h < 0) return fail(NEDNER_E_ARG, "detector area must be finite and >= 0 at index " + std::to_string(m));
    }
  }
  if (v.equi) {
    std::vector<int64_t> nodes(d->m);
    for (int64_t m = 0; m < d->m; ++m) {
      long i[2];
      if (!grid_node(*d, v, m, i))
        return fail(NEDNER_E_ARG, "sensor " + std::to_string(m) + " is not on a grid node (NEDNER_EQUISPACED)");
      nodes[m] = int64_t(i[0]) * d->n2 + i[1];
    }
    std::sort(nodes.begin(), nodes.end());
    if (std::adjacent_find(nodes.begin(), nodes.end()) != nodes.end())
      return fail(NEDNER_E_ARG, "two sensors on one grid node (NEDNER_EQUISPACED)");
  }
  // frequencies: |omega| dt over the mode set (both Nyquist representatives)
  {
    // (a single voxel across the second axis has only the mode k2 = 0)
    const double k1 = M_PI * d->n1 / v.L1, k2 = d->n2 == 1 ? 0.0 : M_PI * d->n2 / v.L2;
    const double kz = M_PI * d->n3 / (d->n3 * v.D3);
    v.max_theta = d->c * d->dt * std::sqrt(k1 * k1 + k2 * k2 + kz * kz);
  }
  // supported transform sizes
  for (long n : {v.n1, v.n2, v.ntt, (long)d->n1, (long)d->n2, (long)d->n3})
    if (!five_smooth(n))
      return fail(NEDNER_E_UNSUPPORTED, "FFT length " + std::to_string(n) + " is not 5-smooth (2^a 3^b 5^c)");
  const long lat_max = d->prec == NEDNER_FP64 ? 2048 : 4096;
  if (v.n1 > lat_max || v.n2 > lat_max || d->n1 > lat_max || d->n2 > lat_max)
    return fail(NEDNER_E_UNSUPPORTED, "lateral transform longer than " + std::to_string(lat_max));
  if (column_lds(*d, v) > 160 * 1024)
    return fail(NEDNER_E_UNSUPPORTED, "time FFT length and depth count exceed the LDS of one workgroup");
  // one wavefront transforms a column in place, at most 64 points per lane
  if (v.ntt > 4096 || d->n3 > 4096)
    return fail(NEDNER_E_UNSUPPORTED, "time FFT length or depth count above 4096");
  // spreading launch shape
  int TT = d->time_per_lane;
  if (TT == 0) TT = (d->nt >= 512 && d->nt % 4 == 0) ? 4 : (d->nt >= 128 ? 2 : 1);
  if (d->nt % TT) return fail(NEDNER_E_ARG, "time_per_lane must divide nt");
  v.TT = TT;
  v.nchunk = int((d->nt + 64 * TT - 1) / (64 * TT));
  int S = d->rows_per_wave;
  // default mean sweep length: as long as the launch still has about 1024
  // workgroups (four per CU) to spread over the chip, between 2W and
  // max(4W, n1/4): shorter sweeps spend much of their work on the W-1 warm-up
  // cells, longer ones leave too few wavefronts to hide the load latency
  // (measured on the 128^2 x 512, 256^2 x 1024 and 1024-sensor line
  // workloads; the autotuner refines it)
  if (S == 0) {
    const long fill = long(v.n1) * ((v.n2 + 3) / 4) * v.nchunk / 1024;
    S = int(std::min<long>(std::max<long>(fill, 2L * v.W), std::max<long>(4L * v.W, v.n1 / 4)));
  }
  S = int(std::min<long>(S, v.n1));
  v.S = S;
  v.nseg = int((v.n1 + S - 1) / S);
  v.CB = S + v.W;
  if (out) *out = v;
  if (v.max_theta >= M_PI && !(d->flags & NEDNER_ALLOW_ALIAS))
    return fail(NEDNER_E_ALIAS, "max |omega| dt = " + std::to_string(v.max_theta) +
                                    " >= pi: time sampling aliases (set NEDNER_ALLOW_ALIAS to accept)");
  return NEDNER_OK;
}

// Host geometry shared by the query and the plan.
struct Geometry {
  std::vector<int> cell;        // [M][2]
  std::vector<double> w1, w2;   // [M][W]
  std::vector<double> w1u;      // [M][W] first-axis window values without s_m
  std::vector<int> ent_m;
  std::vector<double> ent_w2;
  std::vector<int> cellbeg;     // per segment, per column of its group: list offsets per sweep cell
  std::vector<int> segd;        // [segments][4]: column group, first row S0, end row S1, offset of
                                // the group's first column's table in cellbeg
  std::vector<int> node;        // equispaced: [n1 * n2] sensor at each node, -1 where none
  std::vector<double> s;        // equispaced: [M] h_m / (d1 d2)
};

void build_geometry(const nedner_desc& d, const Derived& v, Geometry& G) {
  const int64_t M = d.m;
  if (v.equi) {
    G.cell.resize(2 * M);
    G.s.resize(M);
    G.node.assign((size_t)d.n1 * d.n2, -1);
    for (int64_t m = 0; m < M; ++m) {
      long i[2] = {0, 0};
      grid_node(d, v, m, i);
      G.cell[2 * m] = int(i[0]);
      G.cell[2 * m + 1] = int(i[1]);
      G.s[m] = (d.h ? d.h[m] : v.L1 * v.L2 / double(M)) / (d.d1 * d.d2);
      G.node[(size_t)i[0] * d.n2 + i[1]] = int(m);
    }
    return;
  }
  const int W = v.W, h = W / 2 - 1;
  const bool plain = d.prec == NEDNER_FP32_PLAIN;
  G.cell.resize(2 * M);
  G.w1.resize(M * W);
  G.w1u.resize(M * W);
  G.w2.resize(M * W);
  std::vector<double> frac2(M);
  const double L[2] = {v.L1, v.L2}, a[2] = {d.a1, d.a2};
  const long n[2] = {v.n1, v.n2};
  for (int64_t m = 0; m < M; ++m) {
    const double s = (d.h ? d.h[m] : v.L1 * v.L2 / double(M)) / (d.d1 * d.d2);
    for (int ax = 0; ax < 2; ++ax) {
      double u, f;
      long c;
      if (plain) {
        float uf = float(n[ax]) * (float(d.xy[2 * m + ax]) - float(a[ax])) / float(L[ax]);
        uf -= float(n[ax]) * std::floor(uf / float(n[ax]));
        if (uf >= float(n[ax])) uf -= float(n[ax]);
        const float cf = std::floor(uf);
        c = long(cf);
        f = double(uf - cf);
        u = uf;
      } else {
        u = double(n[ax]) * (d.xy[2 * m + ax] - a[ax]) / L[ax];
        u -= double(n[ax]) * std::floor(u / double(n[ax]));
        if (u >= double(n[ax])) u -= double(n[ax]);
        c = long(std::floor(u));
        f = u - double(c);
      }
      (void)u;
      G.cell[2 * m + ax] = int(c);
      for (int k = 0; k < W; ++k) {
        const int o = k - h;
        double w;
        if (plain) {
          const float df = float(o) - float(f);
          w = v.window == NEDNER_WINDOW_GAUSSIAN ? double(std::exp(-float(v.beta) * df * df))
                                                 : double(float(window_phi(v, double(df))));
        } else {
          w = window_phi(v, double(o) - f);
        }
        if (ax == 0) {
          G.w1[m * W + k] = s * w;
          G.w1u[m * W + k] = w;
        } else
          G.w2[m * W + k] = w;
      }
      if (ax == 1) frac2[m] = f;
    }
  }
  // per-column lists: sensors whose second-axis taps reach column q2
  struct E {
    int c1, m;
    double w2;
  };
  std::vector<std::vector<E>> percol(v.n2);
  std::vector<std::pair<int, double>> taps;
  for (int64_t m = 0; m < M; ++m) {
    taps.clear();
    for (int k = 0; k < W; ++k) {
      const int q2 = int(((long)G.cell[2 * m + 1] + k - h) % v.n2 + v.n2) % int(v.n2);
      const double w = G.w2[m * W + k];
      bool merged = false;
      for (auto& t : taps)
        if (t.first == q2) {
          t.second += w;
          merged = true;
        }
      if (!merged) taps.push_back({q2, w});
    }
    for (auto& t : taps) percol[t.first].push_back({G.cell[2 * m], int(m), t.second});
  }
  // each column's entries sorted by first-axis cell (counting sort, stable:
  // sensor order within a cell)
  std::vector<std::vector<int>> rowstart(v.n2);
  std::vector<std::vector<E>> sorted(v.n2);
  int64_t total = 0;
  for (long q2 = 0; q2 < v.n2; ++q2) {
    auto& L2v = percol[q2];
    auto& rs = rowstart[q2];
    rs.assign(v.n1 + 1, 0);
    for (auto& e : L2v) rs[e.c1 + 1]++;
    for (long r = 0; r < v.n1; ++r) rs[r + 1] += rs[r];
    sorted[q2].resize(L2v.size());
    std::vector<int> pos(rs.begin(), rs.end() - 1);
    for (auto& e : L2v) sorted[q2][pos[e.c1]++] = e;
    total += int64_t(L2v.size());
    std::vector<E>().swap(L2v);
  }
  // Sweep segments, per group of four columns (one workgroup): a segment of
  // rows [S0, S1) sweeps the cell rows S0 - W/2 .. S1 + W/2 - 2, and costs the
  // entries of those cell rows over the group's columns. Segments are cut so
  // that each costs about what a segment of S rows costs at the mean density,
  // W-1 overlap rows included: dense parts of the aperture get short
  // segments, sparse ones long ones, and every wavefront of the launch does
  // about the same work. Segments keep at least min(W, S) rows (shorter ones
  // would mostly sweep overlap) and at most 4 S.
  // NEDNER_SEGMENTS="cut,order" overrides the defaults (cut 0: balanced as
  // above, 1: fixed S rows; order 0: the segments of a group consecutive,
  // 1: by first row, then group).
  int seg_cut = 0, seg_order = 0;
  if (const char* e = getenv("NEDNER_SEGMENTS")) {
    int a = 0, b = 0;
    if (sscanf(e, "%d,%d", &a, &b) == 2) {
      seg_cut = a;
      seg_order = b;
    }
  }
  const long ncg = (v.n2 + 3) / 4;
  const double avg = double(total) / (double(ncg) * double(v.n1));
  const double target = seg_cut == 1 ? 1e300 : avg * double(v.S + W - 1);
  const long minlen = seg_cut == 1 ? std::min<long>(v.S, v.n1) : std::max<long>(1, std::min<long>(W, v.S));
  const long maxlen = seg_cut == 1 ? std::min<long>(v.S, v.n1) : std::min<long>(v.n1, 4L * v.S);
  std::vector<double> cost(v.n1);
  auto rowcost = [&](long V) { return cost[size_t(((V % v.n1) + v.n1) % v.n1)]; };
  G.segd.clear();
  G.cellbeg.clear();
  for (long cg = 0; cg < ncg; ++cg) {
    std::fill(cost.begin(), cost.end(), 0.0);
    for (long w = 0; w < 4 && 4 * cg + w < v.n2; ++w) {
      const auto& rs = rowstart[4 * cg + w];
      for (long r = 0; r < v.n1; ++r) cost[r] += double(rs[r + 1] - rs[r]);
    }
    long S0 = 0;
    while (S0 < v.n1) {
      long S1 = std::min<long>(S0 + minlen, v.n1);
      double c = 0.0;
      for (long V = S0 - W / 2; V <= S1 + W / 2 - 2; ++V) c += rowcost(V);
      while (S1 < v.n1 && S1 - S0 < maxlen) {
        const double add = rowcost(S1 + W / 2 - 1);
        if (c + add > target) break;
        c += add;
        ++S1;
      }
      G.segd.insert(G.segd.end(), {int(cg), int(S0), int(S1), int(G.cellbeg.size())});
      const long len = S1 - S0 + W;  // offsets of cell rows Vstart..Vend, then the end
      for (long w = 0; w < 4; ++w) {
        const long q2 = 4 * cg + w;
        const size_t base = G.cellbeg.size();
        G.cellbeg.resize(base + size_t(len), int(G.ent_m.size()));
        if (q2 >= v.n2) continue;
        const auto& rs = rowstart[q2];
        const auto& so = sorted[q2];
        const long Vstart = S0 - W / 2, Vend = S1 + W / 2 - 2;
        for (long V = Vstart; V <= Vend; ++V) {
          G.cellbeg[base + size_t(V - Vstart)] = int(G.ent_m.size());
          const long c1 = ((V % v.n1) + v.n1) % v.n1;
          for (int i = rs[c1]; i < rs[c1 + 1]; ++i) {
            G.ent_m.push_back(so[i].m);
            G.ent_w2.push_back(so[i].w2);
          }
        }
        G.cellbeg[base + size_t(Vend - Vstart + 1)] = int(G.ent_m.size());
      }
      S0 = S1;
    }
  }
  if (seg_order == 1) {
    const size_t ns = G.segd.size() / 4;
    std::vector<size_t> idx(ns);
    for (size_t i = 0; i < ns; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
      return G.segd[4 * a + 1] != G.segd[4 * b + 1] ? G.segd[4 * a + 1] < G.segd[4 * b + 1]
                                                     : G.segd[4 * a] < G.segd[4 * b];
    });
    std::vector<int> sorted_d(G.segd.size());
    for (size_t i = 0; i < ns; ++i)
      for (int k = 0; k < 4; ++k) sorted_d[4 * i + k] = G.segd[4 * idx[i] + k];
    G.segd.swap(sorted_d);
  }
}

struct DevAlloc {
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  template <typename T>
  const void* upload(const std::vector<T>& h) {
    if (err != hipSuccess) return nullptr;
    void* p = nullptr;
    const size_t b = std::max<size_t>(h.size() * sizeof(T), 16);
    err = hipMalloc(&p, b);
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(p);
    if (!h.empty()) err = hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    return p;
  }
  template <typename T>
  const void* upload_as(const std::vector<double>& h) {
    std::vector<T> t(h.begin(), h.end());
    return upload(t);
  }
  template <typename T>
  const void* twiddles(int n) {
    std::vector<T> t(2 * (size_t)n);
    for (int k = 0; k < n; ++k) {
      const double ang = 2.0 * M_PI * double(k) / double(n);
      t[2 * k] = T(std::cos(ang));
      t[2 * k + 1] = T(-std::sin(ang));
    }
    return upload(t);
  }
};

// Device spreading lists of one geometry. The sensor indices and weights are
// padded with zeros past the end so that the staged sweep may read ahead.
struct ListTables {
  const int* em = nullptr;
  const void* ew = nullptr;
  const int* cb = nullptr;
  const int* segd = nullptr;
  int nsegt = 0;
};
constexpr int LIST_PAD = 16;

ListTables upload_lists(const Geometry& G, bool wide, DevAlloc& L) {
  ListTables t;
  const size_t n = G.ent_m.size();
  std::vector<int> em(G.ent_m);
  em.resize(n + LIST_PAD, 0);
  std::vector<double> ew(G.ent_w2);
  ew.resize(n + LIST_PAD, 0.0);
  t.em = static_cast<const int*>(L.upload(em));
  t.ew = wide ? L.upload(ew) : L.upload_as<float>(ew);
  t.cb = static_cast<const int*>(L.upload(G.cellbeg));
  t.segd = static_cast<const int*>(L.upload(G.segd));
  t.nsegt = int(G.segd.size() / 4);
  return t;
}

}  // namespace

struct nedner_plan_s {
  KP kp{};
  nedner_desc desc{};
  Derived v{};
  nedner_info info{};
  int device = 0;
  bool broken = false;
  std::vector<void*> allocs;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  size_t need_ws = 0;
  size_t off1 = 0;
  std::vector<nedner_plan_s*> subs;  // batched plans
  // unit sensor weights for the forward operator Q: w1 without s_m, and the
  // equispaced placement's weights set to one
  const void* w1_unit = nullptr;
  const void* s_unit = nullptr;
  // batched plan state (subs non-empty)
  nedner::BatchProb* d_bp = nullptr;       // device problem table
  int2* d_items = nullptr;                 // work lists of all stages, concatenated
  int* d_counters = nullptr;               // queue heads: one per stage, then one per column class
  int stage_off[nedner::ST_COUNT] = {};    // offset of each stage's list in d_items
  int stage_total[nedner::ST_COUNT] = {};
  size_t pass_smem[nedner::ST_COUNT] = {};
  // The NER column kernel's shape (wavefronts per column, points per thread)
  // is a compile-time one, set by the transform length: the problems of a
  // batch fall into classes of equal shape, each with its own persistent
  // launch, work list (inside the column stage's list) and queue head.
  struct ColClass {
    KP kp0{};          // largest transform of the class (fixes the launch's shape)
    int cpw = 1;       // columns per workgroup
    size_t smem = 0;   // LDS per workgroup
    int off = 0, total = 0;
    std::vector<int> members;
  };
  std::vector<ColClass> col_classes;
  int ncounters = nedner::ST_COUNT;
  KP kp0{};                                // uniform launch parameters of the batch
  std::vector<size_t> sub_off;             // workspace slice of each problem
  void* d_items_alloc = nullptr;           // current work-list allocation (also in d_items)
  // host copies of the geometry, to rebuild the spreading lists for a new shape
  std::vector<double> hxy, hh;
  std::vector<void*> list_allocs;          // device spreading lists (replaced on reshaping)
  // stage profiling
  std::vector<hipEvent_t> ev;
  int prof_max = 0, prof_runs = 0, prof_stages = 0;
  const char* prof_names = nullptr;
};

namespace {

void fill_info(const nedner_desc& d, const Derived& v, int64_t entries, int64_t segments,
               int64_t cb_entries, nedner_info* info) {
  std::memset(info, 0, sizeof(*info));
  info->n1_os = int(v.n1);
  info->n2_os = int(v.n2);
  info->nt_os = int(v.ntt);
  info->columns = v.J1 * v.K2;
  info->segments = int(segments);
  info->rows_per_wave = v.S;
  info->time_per_lane = v.TT;
  size_t off1;
  workspace_layout(d, v, &off1, &info->workspace_bytes);
  const size_t ws = weight_size(d.prec), rs = real_size(d.prec);
  info->list_entries = entries;
  info->table_bytes = (size_t)d.m * (2 * v.W * ws + 8) + entries * (4 + ws) +
                      size_t(cb_entries) * 4 + size_t(segments) * 16 + (v.J1 + v.K2 + d.nt) * rs +
                      2 * rs * (v.n1 + v.n2 + v.ntt + d.n1 + d.n2 + d.n3);
  info->beta = v.beta;
  info->max_abs_theta = v.max_theta;
}

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    ok_ = hipGetDevice(&old_) == hipSuccess;
    if (ok_ && old_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur;
    if (hipGetDevice(&cur) == hipSuccess && cur != old_) (void)hipSetDevice(old_);
  }
  bool ok() const { return ok_; }

 private:
  int old_ = 0;
  bool ok_ = false;
};

void destroy_one(nedner_plan p);
nedner_status batch_upload_table(nedner_plan bp);
nedner_status forward_impl(nedner_plan plan, const void* d_g, void* d_out, int kind, hipStream_t s,
                           const KP* kp = nullptr);
nedner_status batch_build_lists(nedner_plan bp);
size_t stage_blocks(const KP& k, int stage, int cpw);
bool sweep_gather_ok(const KP& k);
size_t pass_lds(const KP& k, int stage);

nedner_status hip_fail(nedner_plan p, hipError_t e, const char* where) {
  if (p) p->broken = true;
  return fail(NEDNER_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

nedner_status create_one(const nedner_desc* desc_in, int device, nedner_plan* out) {
  Derived v;
  nedner_status st = validate_impl(desc_in, &v);
  if (st != NEDNER_OK) return st;
  nedner_desc dd = *desc_in;
  const nedner_desc* desc = &dd;
  nedner_plan p = new (std::nothrow) nedner_plan_s();
  if (!p) return fail(NEDNER_E_OOM, "host allocation failed");
  p->desc = *desc;
  p->desc.xy = nullptr;
  p->desc.h = nullptr;
  p->v = v;
  p->device = device;
  Geometry G;
  try {
    build_geometry(*desc, v, G);
  } catch (const std::bad_alloc&) {
    delete p;
    return fail(NEDNER_E_OOM, "host allocation failed while building the spreading lists");
  }
  if (G.ent_m.size() > size_t(INT32_MAX)) {
    delete p;
    return fail(NEDNER_E_UNSUPPORTED, "too many spreading list entries");
  }
  fill_info(*desc, v, int64_t(G.ent_m.size()), int64_t(G.segd.size() / 4), int64_t(G.cellbeg.size()),
            &p->info);
  workspace_layout(*desc, v, &p->off1, &p->need_ws);

  DeviceGuard guard(device);
  if (!guard.ok()) {
    delete p;
    return fail(NEDNER_E_HIP, "cannot select device " + std::to_string(device));
  }
  KP& k = p->kp;
  k.M = int(desc->m);
  k.Nt = int(desc->nt);
  k.N1 = desc->n1;
  k.N2 = desc->n2;
  k.N3 = desc->n3;
  k.n1 = int(v.n1);
  k.n2 = int(v.n2);
  k.ntt = int(v.ntt);
  k.K2 = v.K2;
  k.J1 = v.J1;
  k.W = v.W;
  k.TT = v.TT;
  k.S = v.S;
  k.nseg = v.nseg;
  k.CB = v.CB;
  k.nchunk = v.nchunk;
  k.prec = desc->prec;
  k.beta = v.beta;
  k.window = v.window;
  k.cdtnt = desc->c * desc->dt * double(v.ntt);
  k.inv_L1sq = 1.0 / (v.L1 * v.L1);
  k.inv_L2sq = 1.0 / (v.L2 * v.L2);
  k.bz = 1.0 / ((desc->n3 * v.D3) * (desc->n3 * v.D3));
  k.phase_p = (desc->nt / 2.0 + desc->t0 / desc->dt) / double(v.ntt);
  k.two_c = 2.0 * desc->c;
  k.scale_spec = desc->dt / v.D3;
  k.scale_vol = k.scale_spec / (double(desc->n1) * desc->n2 * desc->n3);
  k.r_n1 = make_radices(k.n1);
  k.r_n2 = make_radices(k.n2);
  k.r_ntt = make_radices(k.ntt);
  k.r_N1 = make_radices(k.N1);
  k.r_N2 = make_radices(k.N2);
  k.r_N3 = make_radices(k.N3);

  // deconvolution and precorrection tables
  std::vector<double> d1(v.J1), d2(v.K2), dtb(desc->nt);
  // no lateral window on the equispaced path: the lateral DFT is exact
  for (int je = 0; je < v.J1; ++je) d1[je] = v.equi ? 1.0 : 1.0 / window_phihat(v, je - desc->n1 / 2, double(v.n1));
  for (int k2 = 0; k2 < v.K2; ++k2) d2[k2] = v.equi ? 1.0 : 1.0 / window_phihat(v, k2, double(v.n2));
  for (int64_t n = 0; n < desc->nt; ++n) dtb[n] = 1.0 / window_phihat(v, double(n - desc->nt / 2), double(v.ntt));

  DevAlloc A;
  // FFT pass shape: 16 lines (whole 128-byte rows of float pairs), 512
  // threads, in place (measured best on the 128^2 x 512 and 256^2 x 1024
  // workloads); NEDNER_PASS_SHAPE="lines,threads,inplace" overrides it
  k.pass_lines = 16;
  k.pass_threads = 512;
  k.pass_ip = 1;
  if (const char* e = getenv("NEDNER_PASS_SHAPE")) {
    int a = 0, b = 0, c = 0;
    if (sscanf(e, "%d,%d,%d", &a, &b, &c) == 3 && a > 0 && (a & (a - 1)) == 0 && b >= 64 && b <= 512 &&
        b % 64 == 0) {
      k.pass_lines = a;
      k.pass_threads = b;
      k.pass_ip = c != 0;
    }
  }
  const SpreadOpt so = spread_opt();
  k.spread_pd = so.pd;
  k.wide_w = desc->prec == NEDNER_FP32_WIDE && so.wide;
  const bool wide = desc->prec == NEDNER_FP64 || k.wide_w;
  const bool dbl = desc->prec == NEDNER_FP64;
  k.w1 = wide ? A.upload(G.w1) : A.upload_as<float>(G.w1);
  k.w2 = wide ? A.upload(G.w2) : A.upload_as<float>(G.w2);
  k.cell = static_cast<const int*>(A.upload(G.cell));
  k.equi = v.equi;
  k.cosm = 0;
  if (v.equi) {
    k.node = static_cast<const int*>(A.upload(G.node));
    k.sw = dbl ? A.upload(G.s) : A.upload_as<float>(G.s);
    const std::vector<double> ones(size_t(desc->m), 1.0);
    p->s_unit = dbl ? A.upload(ones) : A.upload_as<float>(ones);
  } else {
    p->w1_unit = wide ? A.upload(G.w1u) : A.upload_as<float>(G.w1u);
    // the adjoint gather's sensor order: by tiles of 4 x 4 cells, then by cell
    std::vector<int> order(size_t(desc->m));
    for (int64_t m = 0; m < desc->m; ++m) order[m] = int(m);
    std::sort(order.begin(), order.end(), [&](int x, int y) {
      const int x1 = G.cell[2 * size_t(x)], x2 = G.cell[2 * size_t(x) + 1];
      const int y1 = G.cell[2 * size_t(y)], y2 = G.cell[2 * size_t(y) + 1];
      if ((x1 >> 2) != (y1 >> 2)) return (x1 >> 2) < (y1 >> 2);
      if ((x2 >> 2) != (y2 >> 2)) return (x2 >> 2) < (y2 >> 2);
      if (x1 != y1) return x1 < y1;
      if (x2 != y2) return x2 < y2;
      return x < y;
    });
    k.gorder = static_cast<const int*>(A.upload(order));
    // the sweep gather's tables: the sensors of each pair of second-axis cell
    // columns (2c, 2c + 1) by first-axis cell (a counting sort: index order
    // within a cell), each entry 2 m + (c2 - 2c)
    const size_t n1 = size_t(v.n1), n2 = size_t(v.n2);
    bool in_grid = true;
    for (int64_t m = 0; m < desc->m && in_grid; ++m)
      in_grid = G.cell[2 * size_t(m)] >= 0 && size_t(G.cell[2 * size_t(m)]) < n1 &&
                G.cell[2 * size_t(m) + 1] >= 0 && size_t(G.cell[2 * size_t(m) + 1]) < n2;
    if (in_grid) {
      const size_t np2 = (n2 + 1) / 2;
      std::vector<int> start(n1 * np2 + 1, 0), colm(size_t(desc->m));
      for (int64_t m = 0; m < desc->m; ++m)
        start[size_t(G.cell[2 * size_t(m) + 1] / 2) * n1 + size_t(G.cell[2 * size_t(m)]) + 1]++;
      for (size_t i = 0; i < n1 * np2; ++i) start[i + 1] += start[i];
      // the bounds table is padded by GPAD entries before and after (the
      // sweep reads the bounds of whole blocks of cell rows, which reach past
      // a column's range), the sensor table by two entries (read ahead)
      constexpr size_t GPAD = 64;
      std::vector<int> beg(np2 * (n1 + 1) + 2 * GPAD, 0);
      for (size_t c2 = 0; c2 < np2; ++c2)
        for (size_t c1 = 0; c1 <= n1; ++c1) beg[GPAD + c2 * (n1 + 1) + c1] = start[c2 * n1 + c1];
      std::vector<int> pos(start.begin(), start.end() - 1);
      for (int64_t m = 0; m < desc->m; ++m) {
        const int c2 = G.cell[2 * size_t(m) + 1];
        colm[size_t(pos[size_t(c2 / 2) * n1 + size_t(G.cell[2 * size_t(m)])]++)] = int(2 * m + (c2 & 1));
      }
      colm.push_back(0);
      colm.push_back(0);
      const int* bdev = static_cast<const int*>(A.upload(beg));
      k.gcolbeg = bdev ? bdev + GPAD : nullptr;
      k.gcolm = static_cast<const int*>(A.upload(colm));
      k.gS = sweep_gather_ok(k) ? 128 : 0;
    }
  }
  {
    DevAlloc Lst;
    const ListTables t = upload_lists(G, wide, Lst);
    k.ent_m = t.em;
    k.ent_w2 = t.ew;
    k.cellbeg = t.cb;
    k.segd = t.segd;
    k.nsegt = t.nsegt;
    p->list_allocs = Lst.ptrs;
    if (Lst.err != hipSuccess && A.err == hipSuccess) A.err = Lst.err;
  }
  p->hxy.assign(desc->xy, desc->xy + 2 * desc->m);
  if (desc->h) p->hh.assign(desc->h, desc->h + desc->m);
  k.dec1 = dbl ? A.upload(d1) : A.upload_as<float>(d1);
  k.dec2 = dbl ? A.upload(d2) : A.upload_as<float>(d2);
  k.dect = dbl ? A.upload(dtb) : A.upload_as<float>(dtb);
  if (dbl) {
    k.tw_n1 = A.twiddles<double>(k.n1);
    k.tw_n2 = A.twiddles<double>(k.n2);
    k.tw_ntt = A.twiddles<double>(k.ntt);
    k.tw_N1 = A.twiddles<double>(k.N1);
    k.tw_N2 = A.twiddles<double>(k.N2);
    k.tw_N3 = A.twiddles<double>(k.N3);
  } else {
    k.tw_n1 = A.twiddles<float>(k.n1);
    k.tw_n2 = A.twiddles<float>(k.n2);
    k.tw_ntt = A.twiddles<float>(k.ntt);
    k.tw_N1 = A.twiddles<float>(k.N1);
    k.tw_N2 = A.twiddles<float>(k.N2);
    k.tw_N3 = A.twiddles<float>(k.N3);
  }
  p->allocs = A.ptrs;
  if (A.err != hipSuccess) {
    const hipError_t e = A.err;
    for (void* q : p->allocs) (void)hipFree(q);
    for (void* q : p->list_allocs) (void)hipFree(q);
    delete p;
    if (e == hipErrorOutOfMemory) return fail(NEDNER_E_OOM, "device allocation of plan tables failed");
    return fail(NEDNER_E_HIP, std::string("plan upload: ") + hipGetErrorString(e));
  }
  *out = p;
  return NEDNER_OK;
}

nedner_status exec_check(nedner_plan plan, int kind, bool adj) {
  if (!plan) return fail(NEDNER_E_ARG, "plan is NULL");
  if (plan->broken) return fail(NEDNER_E_STATE, "plan is unusable after an earlier HIP error");
  if (!plan->subs.empty()) return fail(NEDNER_E_ARG, "batched plan: use nedner_execute_many");
  if (kind < 0 || kind > 2) return fail(NEDNER_E_ARG, "unknown kind");
  if (adj && kind == NEDNER_SPECTRUM_COMPLEX)
    return fail(NEDNER_E_UNSUPPORTED, "adjoint of the spectrum output is not provided");
  if (kind != NEDNER_STAGE_GRID && (!plan->ws || plan->ws_bytes < plan->need_ws))
    return fail(NEDNER_E_WORKSPACE, "no workspace, or one smaller than nedner_workspace_size");
  return NEDNER_OK;
}

#define NEDNER_RUN(call, what)                      \
  do {                                              \
    hipError_t e_ = (call);                         \
    if (e_ != hipSuccess) return hip_fail(plan, e_, what); \
  } while (0)

// Records one event before every stage and one after the last, when the plan
// is profiling and has event slots left for this run.
struct Marks {
  nedner_plan plan;
  hipStream_t s;
  int run = -1, stages = 0, next = 0;
  Marks(nedner_plan p, hipStream_t st, int nstages, const char* names) : plan(p), s(st), stages(nstages) {
    if (p->prof_max > 0 && p->prof_runs < p->prof_max) {
      if (p->prof_runs == 0) {
        p->prof_stages = nstages;
        p->prof_names = names;
      }
      if (p->prof_stages == nstages) run = p->prof_runs++;
    }
  }
  hipError_t mark() {
    if (run < 0 || next > stages) return hipSuccess;
    return hipEventRecord(plan->ev[(size_t)run * (stages + 1) + next++], s);
  }
};

static const char* kFwdNames = "spread,lat_a,lat_b,column,pass_c,pass_d";
static const char* kSpecNames = "spread,lat_a,lat_b,column_spectrum";
static const char* kAdjNames = "adj_d,adj_c,column_adj,adj_b,adj_a,gather";

// kp: launch parameters other than the plan's own (the forward operator Q).
nedner_status forward_impl(nedner_plan plan, const void* d_g, void* d_out, int kind, hipStream_t s,
                           const KP* kp) {
  const KP& k = kp ? *kp : plan->kp;
  char* b0 = static_cast<char*>(plan->ws);
  char* b1 = b0 + plan->off1;
  if (kind == NEDNER_STAGE_GRID) {
    Marks mk(plan, s, 1, "spread");
    NEDNER_RUN(mk.mark(), "event");
    NEDNER_RUN(k.equi ? nedner::launch_place(k, d_g, d_out, s) : nedner::launch_spread(k, d_g, d_out, s), "spread");
    NEDNER_RUN(mk.mark(), "event");
    return NEDNER_OK;
  }
  const bool spec = kind == NEDNER_SPECTRUM_COMPLEX;
  Marks mk(plan, s, spec ? 4 : 6, spec ? kSpecNames : kFwdNames);
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(k.equi ? nedner::launch_place(k, d_g, b0, s) : nedner::launch_spread(k, d_g, b0, s), "spread");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_lat_a(k, b0, b1, s), "lateral FFT (second axis)");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_lat_b(k, b1, b0, s), "lateral FFT (first axis)");
  NEDNER_RUN(mk.mark(), "event");
  if (spec) {
    NEDNER_RUN(nedner::launch_column(k, b0, d_out, 1, s), "NER column");
    NEDNER_RUN(mk.mark(), "event");
    return NEDNER_OK;
  }
  NEDNER_RUN(nedner::launch_column(k, b0, b1, 0, s), "NER column");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_pass_c(k, b1, b0, s), "inverse FFT (first axis)");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_pass_d(k, b0, d_out, s), "inverse FFT (second axis)");
  NEDNER_RUN(mk.mark(), "event");
  return NEDNER_OK;
}

nedner_status adjoint_impl(nedner_plan plan, const void* d_in, int kind, void* d_g, hipStream_t s,
                           const KP* kp = nullptr) {
  const KP& k = kp ? *kp : plan->kp;
  char* b0 = static_cast<char*>(plan->ws);
  char* b1 = b0 + plan->off1;
  if (kind == NEDNER_STAGE_GRID) {
    Marks mk(plan, s, 1, "gather");
    NEDNER_RUN(mk.mark(), "event");
    NEDNER_RUN(k.equi ? nedner::launch_place_adj(k, d_in, d_g, s) : nedner::launch_gather(k, d_in, d_g, s), "gather");
    NEDNER_RUN(mk.mark(), "event");
    return NEDNER_OK;
  }
  Marks mk(plan, s, 6, kAdjNames);
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_adj_d(k, d_in, b0, s), "adjoint FFT (second axis)");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_adj_c(k, b0, b1, s), "adjoint FFT (first axis)");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_column_adj(k, b1, b0, s), "adjoint NER column");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_adj_b(k, b0, b1, s), "adjoint lateral FFT (first axis)");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_adj_a(k, b1, b0, s), "adjoint lateral FFT (second axis)");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(k.equi ? nedner::launch_place_adj(k, b0, d_g, s) : nedner::launch_gather(k, b0, d_g, s), "gather");
  NEDNER_RUN(mk.mark(), "event");
  return NEDNER_OK;
}

// Launch parameters of the forward operator Q of the wave equation (Sec. 2)
// and of its adjoint: the adjoint and forward pipelines of the plan with unit
// sensor weights, the constant weight 1/(N1 N2 N3) in place of (dt/d3) W(j,l),
// and the l, -l average of the NER column values.
KP trace_params(const nedner_plan p) {
  KP k = p->kp;
  if (k.equi)
    k.sw = p->s_unit;
  else
    k.w1 = p->w1_unit;
  k.scale_vol = 1.0 / (double(k.N1) * double(k.N2) * double(k.N3));
  k.cosm = 1;
  return k;
}

// ---------------------------------------------------------------- batches

size_t stage_blocks(const KP& k, int stage, int cpw) {
  auto ceil_div = [](long a, long b) { return (a + b - 1) / b; };
  const int cs = k.prec == NEDNER_FP64 ? 16 : 8;
  switch (stage) {
    case nedner::ST_SPREAD: {
      const long G = (long)k.nsegt * k.nchunk;
      return size_t(8 * ceil_div(G, 8));
    }
    case nedner::ST_LAT_A: return size_t(ceil_div(k.Nt / 2, nedner::pass_lines_for(k, k.n2, cs)) * k.n1);
    case nedner::ST_LAT_B: return size_t(ceil_div(k.Nt, nedner::pass_lines_for(k, k.n1, cs)) * k.K2);
    case nedner::ST_COLUMN: return size_t(ceil_div((long)k.J1 * k.K2, cpw));
    case nedner::ST_PASS_C: return size_t(ceil_div(k.N3, nedner::pass_lines_for(k, k.N1, cs)) * k.K2);
    default: return size_t(ceil_div(k.N3 / 2, nedner::pass_lines_for(k, k.N2, cs)) * k.N1);
  }
}

size_t pass_lds(const KP& k, int stage) {
  const int cs = k.prec == NEDNER_FP64 ? 16 : 8;
  int n = 0;
  switch (stage) {
    case nedner::ST_LAT_A: n = k.n2; break;
    case nedner::ST_LAT_B: n = k.n1; break;
    case nedner::ST_PASS_C: n = k.N1; break;
    case nedner::ST_PASS_D: n = k.N2; break;
    default: return 0;
  }
  const int tb = nedner::pass_lines_for(k, n, cs);
  return (size_t)n * cs * ((k.pass_ip ? 1 : 2) * (size_t)tb + 1);
}

nedner_status create_batch(const nedner_desc* descs, int count, int device, nedner_plan* out) {
  if (!descs || count < 1 || count > 4096) return fail(NEDNER_E_ARG, "count must be in [1, 4096]");
  const int prec = descs[0].prec, w = descs[0].w;
  bool all4 = true;
  for (int i = 0; i < count; ++i) {
    if (descs[i].prec != prec || descs[i].w != w || descs[i].window != descs[0].window)
      return fail(NEDNER_E_ARG, "all problems of a batch must share precision, window and window width");
    if (descs[i].flags & NEDNER_EQUISPACED)
      return fail(NEDNER_E_UNSUPPORTED, "batched plans do not take NEDNER_EQUISPACED");
    if (descs[i].nt % 4) all4 = false;
  }
  // the spreading kernel's time-per-lane is a compile-time shape: one for the batch
  int TT = descs[0].time_per_lane;
  if (TT == 0) TT = all4 ? 4 : 2;
  nedner_plan bp = new (std::nothrow) nedner_plan_s();
  if (!bp) return fail(NEDNER_E_OOM, "host allocation failed");
  bp->device = device;
  for (int i = 0; i < count; ++i) {
    nedner_desc d = descs[i];
    d.time_per_lane = TT;
    // the problems of a batch share the chip: long sweeps (less overlap work)
    // beat the short ones a problem alone needs to fill it (the batch
    // autotuner picks 256 rows, clamped to each grid, on the 64-problem set)
    if (d.rows_per_wave == 0) d.rows_per_wave = 256;
    nedner_plan sp = nullptr;
    nedner_status st = create_one(&d, device, &sp);
    if (st != NEDNER_OK) {
      const std::string msg = "problem " + std::to_string(i) + ": " + g_last_error;
      destroy_one(bp);
      return fail(st, msg);
    }
    bp->subs.push_back(sp);
  }
  // uniform launch parameters of the other stages; the column stage by class
  bp->kp0 = bp->subs[0]->kp;
  for (auto* sp : bp->subs) {
    bp->kp0.ntt = std::max(bp->kp0.ntt, sp->kp.ntt);
    bp->kp0.N3 = std::max(bp->kp0.N3, sp->kp.N3);
  }
  for (int i = 0; i < count; ++i) {
    const KP& k = bp->subs[i]->kp;
    const int wpc = nedner::column_wpc_host(k), ppt = nedner::column_ppt_host(k);
    size_t ci = 0;
    while (ci < bp->col_classes.size() && !(nedner::column_wpc_host(bp->col_classes[ci].kp0) == wpc &&
                                            nedner::column_ppt_host(bp->col_classes[ci].kp0) == ppt))
      ++ci;
    if (ci == bp->col_classes.size()) {
      bp->col_classes.emplace_back();
      bp->col_classes.back().kp0 = k;
    }
    auto& c = bp->col_classes[ci];
    c.kp0.ntt = std::max(c.kp0.ntt, k.ntt);
    c.kp0.N3 = std::max(c.kp0.N3, k.N3);
    c.members.push_back(i);
  }
  for (auto& c : bp->col_classes) {
    size_t wave_max = 0, shared_max = 0;
    for (int i : c.members) {
      wave_max = std::max(wave_max, nedner::column_wave_bytes_host(bp->subs[i]->kp));
      shared_max = std::max(shared_max, nedner::column_shared_bytes_host(bp->subs[i]->kp));
    }
    // columns per workgroup (of wpc wavefronts each, at most 512 threads):
    // the most resident wavefronts per CU within its 160 KB of LDS
    const int wpc = nedner::column_wpc_host(c.kp0);
    int best = 1;
    size_t best_waves = 0;
    for (int cw = 1; cw * wpc <= 8; ++cw) {
      const size_t wg = shared_max + cw * wave_max;
      if (wg > 160 * 1024) break;
      const size_t waves = cw * wpc * ((160 * 1024) / wg);
      if (waves > best_waves) {
        best_waves = waves;
        best = cw;
      }
    }
    c.cpw = best;
    c.smem = shared_max + best * wave_max;
  }
  bp->ncounters = nedner::ST_COUNT + int(bp->col_classes.size());
  // workspace slices
  size_t off = 0;
  for (auto* sp : bp->subs) {
    bp->sub_off.push_back(off);
    off += align256(sp->need_ws);
  }
  bp->need_ws = std::max<size_t>(off, 256);
  DeviceGuard guard(device);
  {
    nedner_status ls = batch_build_lists(bp);
    if (ls != NEDNER_OK) {
      const std::string msg = g_last_error;
      destroy_one(bp);
      return fail(ls, msg);
    }
  }
  DevAlloc A;
  std::vector<int> zeros(bp->ncounters, 0);
  bp->d_counters = static_cast<int*>(const_cast<void*>(A.upload(zeros)));
  if (A.err == hipSuccess) {
    void* q = nullptr;
    A.err = hipMalloc(&q, sizeof(nedner::BatchProb) * count);
    if (A.err == hipSuccess) A.ptrs.push_back(q);
    bp->d_bp = static_cast<nedner::BatchProb*>(q);
  }
  bp->allocs.insert(bp->allocs.end(), A.ptrs.begin(), A.ptrs.end());
  if (A.err != hipSuccess) {
    const hipError_t e = A.err;
    destroy_one(bp);
    return fail(e == hipErrorOutOfMemory ? NEDNER_E_OOM : NEDNER_E_HIP,
                std::string("batch tables: ") + hipGetErrorString(e));
  }
  bp->info = bp->subs[0]->info;
  bp->info.workspace_bytes = bp->need_ws;
  *out = bp;
  return NEDNER_OK;
}

// Write the problem table (kernel parameters and workspace slices) to the device.
nedner_status batch_upload_table(nedner_plan bp) {
  std::vector<nedner::BatchProb> t(bp->subs.size());
  char* ws = static_cast<char*>(bp->ws);
  for (size_t i = 0; i < t.size(); ++i) {
    t[i].kp = bp->subs[i]->kp;
    t[i].g = nullptr;
    t[i].out = nullptr;
    t[i].b0 = ws + bp->sub_off[i];
    t[i].b1 = ws + bp->sub_off[i] + bp->subs[i]->off1;
  }
  DeviceGuard guard(bp->device);
  const hipError_t e = hipMemcpy(bp->d_bp, t.data(), t.size() * sizeof(t[0]), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(bp, e, "batch table upload");
  return NEDNER_OK;
}

nedner_status execute_many_impl(nedner_plan plan, const void* const* d_g, void* const* d_out, hipStream_t s) {
  const int count = int(plan->subs.size());
  bool vec = true;
  for (int i = 0; i < count; ++i) {
    if (!d_g[i] || !d_out[i]) return fail(NEDNER_E_ARG, "NULL device pointer for problem " + std::to_string(i));
    const size_t al = (size_t)plan->kp0.TT * (plan->kp0.prec == NEDNER_FP64 ? 8 : 4);
    if (reinterpret_cast<uintptr_t>(d_g[i]) % al) vec = false;
  }
  Marks mk(plan, s, 6, kFwdNames);
  for (int first = 0; first < count; first += 64) {
    nedner::PtrChunk ch{};
    ch.first = first;
    ch.n = std::min(64, count - first);
    for (int i = 0; i < ch.n; ++i) {
      ch.g[i] = d_g[first + i];
      ch.out[i] = d_out[first + i];
    }
    NEDNER_RUN(nedner::launch_batch_prepare(plan->d_bp, ch, plan->d_counters, first == 0 ? plan->ncounters : 0, s),
               "batch prepare");
  }
  auto wl = [&](int st) {
    return nedner::WorkList{plan->d_items + plan->stage_off[st], plan->stage_total[st], plan->d_counters + st};
  };
  const KP& k0 = plan->kp0;
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_spread_many(k0, plan->d_bp, wl(nedner::ST_SPREAD), vec, s), "batched spread");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_pass_many(k0, nedner::ST_LAT_A, plan->d_bp, wl(nedner::ST_LAT_A),
                                      plan->pass_smem[nedner::ST_LAT_A], s), "batched lateral FFT");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_pass_many(k0, nedner::ST_LAT_B, plan->d_bp, wl(nedner::ST_LAT_B),
                                      plan->pass_smem[nedner::ST_LAT_B], s), "batched lateral FFT");
  NEDNER_RUN(mk.mark(), "event");
  for (size_t ci = 0; ci < plan->col_classes.size(); ++ci) {
    const auto& c = plan->col_classes[ci];
    const nedner::WorkList cl{plan->d_items + plan->stage_off[nedner::ST_COLUMN] + c.off, c.total,
                              plan->d_counters + nedner::ST_COUNT + ci};
    NEDNER_RUN(nedner::launch_column_many(c.kp0, plan->d_bp, cl, c.cpw, c.smem, s), "batched NER column");
  }
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_pass_many(k0, nedner::ST_PASS_C, plan->d_bp, wl(nedner::ST_PASS_C),
                                      plan->pass_smem[nedner::ST_PASS_C], s), "batched inverse FFT");
  NEDNER_RUN(mk.mark(), "event");
  NEDNER_RUN(nedner::launch_pass_many(k0, nedner::ST_PASS_D, plan->d_bp, wl(nedner::ST_PASS_D),
                                      plan->pass_smem[nedner::ST_PASS_D], s), "batched inverse FFT");
  NEDNER_RUN(mk.mark(), "event");
  return NEDNER_OK;
}

// ---------------------------------------------------------------- reshaping and tuning

// Rebuild the spreading lists of a single-problem plan for sweeps of S rows
// and TT samples per lane (PD, the sweep variant, is 1: samples staged
// through LDS). Weights and workspace do not change.
nedner_status set_spread_shape(nedner_plan p, int S, int TT, int PD) {
  nedner_desc d = p->desc;
  d.xy = p->hxy.data();
  d.h = p->hh.empty() ? nullptr : p->hh.data();
  d.rows_per_wave = S;
  d.time_per_lane = TT;
  Derived v;
  nedner_status st = validate_impl(&d, &v);
  if (st != NEDNER_OK) return st;
  Geometry G;
  try {
    build_geometry(d, v, G);
  } catch (const std::bad_alloc&) {
    return fail(NEDNER_E_OOM, "host allocation failed while building the spreading lists");
  }
  DeviceGuard guard(p->device);
  DevAlloc L;
  const bool wide = p->kp.prec == NEDNER_FP64 || p->kp.wide_w;
  const ListTables t = upload_lists(G, wide, L);
  if (L.err != hipSuccess) {
    for (void* q : L.ptrs) (void)hipFree(q);
    return fail(L.err == hipErrorOutOfMemory ? NEDNER_E_OOM : NEDNER_E_HIP,
                std::string("spreading list upload: ") + hipGetErrorString(L.err));
  }
  for (void* q : p->list_allocs) (void)hipFree(q);
  p->list_allocs = L.ptrs;
  KP& k = p->kp;
  k.ent_m = t.em;
  k.ent_w2 = t.ew;
  k.cellbeg = t.cb;
  k.segd = t.segd;
  k.nsegt = t.nsegt;
  k.TT = v.TT;
  k.S = v.S;
  k.nseg = v.nseg;
  k.CB = v.CB;
  k.nchunk = v.nchunk;
  k.spread_pd = PD;
  p->v = v;
  p->desc.rows_per_wave = S;
  p->desc.time_per_lane = TT;
  p->info.segments = t.nsegt;
  p->info.rows_per_wave = v.S;
  p->info.time_per_lane = v.TT;
  p->info.list_entries = int64_t(G.ent_m.size());
  return NEDNER_OK;
}

// Work lists of a batch: per stage, the problems in decreasing order of
// their block count, each problem's blocks consecutive; the column stage's
// list is the concatenation of its classes' lists, each ordered the same way.
nedner_status batch_build_lists(nedner_plan bp) {
  std::vector<int2> items;
  const int count = int(bp->subs.size());
  auto append = [&](const std::vector<int>& probs, int st, int cpw) {
    std::vector<std::pair<size_t, int>> order;
    for (int i : probs) order.push_back({stage_blocks(bp->subs[i]->kp, st, cpw), i});
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<size_t, int>& a, const std::pair<size_t, int>& b) { return a.first > b.first; });
    for (auto& o : order)
      for (size_t b = 0; b < o.first; ++b) items.push_back(make_int2(o.second, int(b)));
  };
  std::vector<int> all(count);
  for (int i = 0; i < count; ++i) all[i] = i;
  for (int st = 0; st < nedner::ST_COUNT; ++st) {
    size_t lds = 0;
    for (int i = 0; i < count; ++i) lds = std::max(lds, pass_lds(bp->subs[i]->kp, st));
    bp->stage_off[st] = int(items.size());
    if (st == nedner::ST_COLUMN) {
      for (auto& c : bp->col_classes) {
        c.off = int(items.size()) - bp->stage_off[st];
        append(c.members, st, c.cpw);
        c.total = int(items.size()) - bp->stage_off[st] - c.off;
      }
    } else {
      append(all, st, 1);
    }
    bp->stage_total[st] = int(items.size()) - bp->stage_off[st];
    bp->pass_smem[st] = lds;
  }
  DeviceGuard guard(bp->device);
  DevAlloc A;
  void* it = const_cast<void*>(A.upload(items));
  if (A.err != hipSuccess) {
    for (void* q : A.ptrs) (void)hipFree(q);
    return fail(NEDNER_E_OOM, std::string("work list upload: ") + hipGetErrorString(A.err));
  }
  if (bp->d_items_alloc) {
    (void)hipFree(bp->d_items_alloc);
    bp->allocs.erase(std::remove(bp->allocs.begin(), bp->allocs.end(), bp->d_items_alloc), bp->allocs.end());
  }
  bp->d_items_alloc = it;
  bp->allocs.push_back(it);
  bp->d_items = static_cast<int2*>(it);
  return NEDNER_OK;
}

bool sweep_gather_ok(const KP& k) {
  // a grid row's samples are addressed with 32-bit byte offsets
  return k.prec != NEDNER_FP64 && k.W <= 12 && k.gcolbeg && k.gcolm && !k.equi &&
         (int64_t)k.n2 * k.Nt * 4 < (int64_t(1) << 31);
}

void get_tuning(nedner_plan p, nedner_tuning* t) {
  std::memset(t, 0, sizeof(*t));
  t->rows_per_wave = p->kp.S;
  t->time_per_lane = p->kp.TT;
  t->spread_depth = p->kp.spread_pd;
  t->pass_lines = p->kp.pass_lines;
  t->pass_threads = p->kp.pass_threads;
  t->pass_inplace = p->kp.pass_ip;
  t->gather_rows = p->kp.gS;
}

bool pass_shape_ok(int lines, int threads) {
  return lines > 0 && (lines & (lines - 1)) == 0 && lines <= 64 && threads >= 64 && threads <= 512 &&
         threads % 64 == 0;
}

// Mean milliseconds of `reps` forward executes of `kind` after one warm-up.
nedner_status time_forward(nedner_plan p, const void* d_g, void* d_out, int kind, hipStream_t s, int reps,
                           double* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return fail(NEDNER_E_HIP, "hipEventCreate failed");
  }
  nedner_status st = forward_impl(p, d_g, d_out, kind, s);
  if (st == NEDNER_OK && hipEventRecord(a, s) != hipSuccess) st = fail(NEDNER_E_HIP, "hipEventRecord failed");
  for (int r = 0; r < reps && st == NEDNER_OK; ++r) st = forward_impl(p, d_g, d_out, kind, s);
  float t = 0.f;
  if (st == NEDNER_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                          hipEventElapsedTime(&t, a, b) != hipSuccess))
    st = fail(NEDNER_E_HIP, "event timing failed");
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = t / reps;
  return st;
}

// Spreading shape search of one problem; U is a buffer of the spread grid's size.
nedner_status tune_spread(nedner_plan p, const void* d_g, void* U, hipStream_t s, int fixed_tt, double* best_ms) {
  const int n1 = p->kp.n1, W = p->kp.W, Nt = p->kp.Nt;
  std::vector<int> tts;
  if (fixed_tt)
    tts.push_back(fixed_tt);
  else
    for (int tt : {4, 2, 1})
      if (Nt % tt == 0 && (tt == 1 || Nt >= 32 * tt) && (tt > 1 || Nt < 128)) tts.push_back(tt);
  // mean sweep lengths on a geometric ladder from 2W to the grid
  std::vector<int> ss;
  for (int S : {24, 32, 48, 64, 96, 128, 171, 256})
    if (S >= 2 * W && S <= n1) ss.push_back(S);
  const int top = std::min(n1, 256);
  if (ss.empty() || ss.back() < top) ss.push_back(top);
  int bS = p->kp.S, bT = p->kp.TT, bP = p->kp.spread_pd;
  double best = 1e300;
  for (int tt : tts)
    for (int S : ss)
      for (int pd : {1}) {
        nedner_status st = set_spread_shape(p, S, tt, pd);
        if (st != NEDNER_OK) return st;
        double ms = 0;
        st = time_forward(p, d_g, U, NEDNER_STAGE_GRID, s, 3, &ms);
        if (st != NEDNER_OK) return st;
        if (ms < best) {
          best = ms;
          bS = S;
          bT = tt;
          bP = pd;
        }
      }
  *best_ms = best;
  return set_spread_shape(p, bS, bT, bP);
}

// Sweep segment length of the adjoint gather: its launch alone on the spread
// grid in U (the values do not change the cost), into a scratch data array.
nedner_status tune_gather(nedner_plan p, const void* U, hipStream_t s) {
  KP& k = p->kp;
  if (!sweep_gather_ok(k)) return NEDNER_OK;
  void* gtmp = nullptr;
  if (hipMalloc(&gtmp, (size_t)k.M * k.Nt * 4) != hipSuccess) return fail(NEDNER_E_OOM, "autotune: no memory");
  hipEvent_t a = nullptr, b = nullptr;
  nedner_status st = NEDNER_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) st = fail(NEDNER_E_HIP, "hipEventCreate failed");
  int best_rows = k.gS;
  double best = 1e300;
  for (int rows : {32, 64, 128, 256, 512}) {
    if (st != NEDNER_OK) break;
    if (rows > k.n1 && rows != 32) break;  // one segment per column already
    k.gS = rows;
    hipError_t e = nedner::launch_gather(k, U, gtmp, s);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = nedner::launch_gather(k, U, gtmp, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (e != hipSuccess) {
      st = hip_fail(p, e, "gather autotune");
      break;
    }
    if (t < best) {
      best = t;
      best_rows = rows;
    }
  }
  k.gS = best_rows;
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(gtmp);
  return st;
}

nedner_status autotune_single(nedner_plan p, const void* d_g, hipStream_t s, nedner_tuning* out) {
  if (!p->ws || p->ws_bytes < p->need_ws) return fail(NEDNER_E_WORKSPACE, "autotune needs the workspace");
  if (!d_g) return fail(NEDNER_E_ARG, "autotune needs a data array");
  double ms_spread = 0;
  nedner_status st = p->kp.equi ? NEDNER_OK : tune_spread(p, d_g, p->ws, s, 0, &ms_spread);
  if (st != NEDNER_OK) return st;
  // the grid of the last spreading run is in the workspace: the gather's input
  st = p->kp.equi ? NEDNER_OK : tune_gather(p, p->ws, s);
  if (st != NEDNER_OK) return st;
  void* vol = nullptr;
  const size_t vb = (size_t)p->kp.N1 * p->kp.N2 * p->kp.N3 * (p->kp.prec == NEDNER_FP64 ? 8 : 4);
  if (hipMalloc(&vol, vb) != hipSuccess) return fail(NEDNER_E_OOM, "autotune: no memory for a volume");
  const int cand[][3] = {{16, 512, 1}, {32, 512, 1}, {8, 512, 1}, {16, 256, 1}, {32, 256, 1},
                         {8, 256, 1},  {16, 256, 0}, {8, 256, 0}, {16, 512, 0}};
  KP& k = p->kp;
  int bl = k.pass_lines, bt = k.pass_threads, bi = k.pass_ip;
  double best = 1e300;
  for (auto& c : cand) {
    k.pass_lines = c[0];
    k.pass_threads = c[1];
    k.pass_ip = c[2];
    double ms = 0;
    st = time_forward(p, d_g, vol, NEDNER_VOLUME_REAL, s, 3, &ms);
    if (st != NEDNER_OK) break;
    if (ms < best) {
      best = ms;
      bl = c[0];
      bt = c[1];
      bi = c[2];
    }
  }
  (void)hipFree(vol);
  k.pass_lines = bl;
  k.pass_threads = bt;
  k.pass_ip = bi;
  if (st != NEDNER_OK) return st;
  if (out) {
    get_tuning(p, out);
    out->ms_spread = ms_spread;
    out->ms_execute = best;
  }
  return NEDNER_OK;
}

// Batched spreading shape: one sweep length for every problem (clamped to its
// grid) and one sweep variant, chosen by timing the whole batch's spreading
// launch on zero data. Problems share the chip in the batch, so the shape that
// is fastest for a problem alone (short sweeps, to fill the chip) is not the
// one that is fastest for the batch (long sweeps, less overlap work).
nedner_status autotune_batch(nedner_plan bp, hipStream_t s, nedner_tuning* out) {
  if (!bp->ws || bp->ws_bytes < bp->need_ws) return fail(NEDNER_E_WORKSPACE, "autotune needs the workspace");
  const int count = int(bp->subs.size());
  // each problem's data: zeros in the second buffer of its workspace slice
  // (the cost does not depend on the values); its first buffer takes the grid
  std::vector<const void*> gz(count);
  std::vector<void*> oz(count);
  for (int i = 0; i < count; ++i) {
    nedner_plan sp = bp->subs[i];
    char* slice = static_cast<char*>(bp->ws) + bp->sub_off[i];
    const size_t gbytes = (size_t)sp->kp.M * sp->kp.Nt * (sp->kp.prec == NEDNER_FP64 ? 8 : 4);
    if (gbytes > sp->need_ws - sp->off1) return fail(NEDNER_E_UNSUPPORTED, "problem data larger than its buffer");
    if (hipMemsetAsync(slice + sp->off1, 0, gbytes, s) != hipSuccess)
      return fail(NEDNER_E_HIP, "hipMemsetAsync failed");
    gz[i] = slice + sp->off1;
    oz[i] = slice;
  }
  auto prepare = [&]() -> hipError_t {
    for (int first = 0; first < count; first += 64) {
      nedner::PtrChunk ch{};
      ch.first = first;
      ch.n = std::min(64, count - first);
      for (int i = 0; i < ch.n; ++i) {
        ch.g[i] = gz[first + i];
        ch.out[i] = oz[first + i];
      }
      hipError_t e = nedner::launch_batch_prepare(bp->d_bp, ch, bp->d_counters, first == 0 ? bp->ncounters : 0, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  auto shape = [&](int S, int pd) -> nedner_status {
    for (auto* sp : bp->subs) {
      nedner_status st = set_spread_shape(sp, std::min<int>(S, sp->kp.n1), bp->kp0.TT, pd);
      if (st != NEDNER_OK) return st;
    }
    bp->kp0.spread_pd = pd;
    nedner_status st = batch_build_lists(bp);
    if (st != NEDNER_OK) return st;
    return batch_upload_table(bp);
  };
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return fail(NEDNER_E_HIP, "hipEventCreate failed");
  }
  double best = 1e300;
  int bS = 64, bP = 1;
  nedner_status st = NEDNER_OK;
  for (int pd : {1}) {
    for (int S : {32, 64, 128, 256}) {
      st = shape(S, pd);
      if (st != NEDNER_OK) break;
      const auto wl = nedner::WorkList{bp->d_items + bp->stage_off[nedner::ST_SPREAD],
                                       bp->stage_total[nedner::ST_SPREAD], bp->d_counters + nedner::ST_SPREAD};
      double ms = 0;
      for (int rep = 0; rep < 3 && st == NEDNER_OK; ++rep) {
        hipError_t e = prepare();
        if (e == hipSuccess) e = hipEventRecord(a, s);
        if (e == hipSuccess) e = nedner::launch_spread_many(bp->kp0, bp->d_bp, wl, 1, s);
        if (e == hipSuccess) e = hipEventRecord(b, s);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
        if (e != hipSuccess) st = hip_fail(bp, e, "batched autotune");
        if (rep > 0) ms += t / 2.0;  // the first launch warms up
      }
      if (st != NEDNER_OK) break;
      if (ms < best) {
        best = ms;
        bS = S;
        bP = pd;
      }
    }
    if (st != NEDNER_OK) break;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st != NEDNER_OK) return st;
  st = shape(bS, bP);
  if (st != NEDNER_OK) return st;
  if (out) {
    get_tuning(bp->subs[0], out);
    out->rows_per_wave = bS;
    out->ms_spread = best;
    out->ms_execute = 0;
  }
  return NEDNER_OK;
}

void free_events(nedner_plan p) {
  for (hipEvent_t e : p->ev) (void)hipEventDestroy(e);
  p->ev.clear();
  p->prof_max = p->prof_runs = p->prof_stages = 0;
}

void destroy_one(nedner_plan p) {
  if (!p) return;
  for (auto* s : p->subs) destroy_one(s);
  if (!p->allocs.empty() || !p->ev.empty() || !p->list_allocs.empty()) {
    DeviceGuard guard(p->device);
    free_events(p);
    for (void* q : p->allocs) (void)hipFree(q);
    for (void* q : p->list_allocs) (void)hipFree(q);
  }
  delete p;
}

}  // namespace

namespace {
nedner_status tenenbaum_impl(const void* d_img, int64_t rows, int64_t cols, int64_t r0, int64_t r1, int64_t c0,
                             int64_t c1, int dtype, bool mean, double* d_result, void* d_work, size_t work_bytes,
                             void* stream) {
  if (!d_img || !d_result || !d_work) return fail(NEDNER_E_ARG, "NULL device pointer");
  if (rows < 1 || cols < 1) return fail(NEDNER_E_ARG, "image sizes must be positive");
  if (r0 < 0 || c0 < 0 || r1 > rows || c1 > cols || r0 > r1 || c0 > c1)
    return fail(NEDNER_E_ARG, "rectangle outside the image");
  if (dtype != NEDNER_DTYPE_F32 && dtype != NEDNER_DTYPE_F64) return fail(NEDNER_E_ARG, "unknown dtype");
  if (work_bytes < nedner::METRICS_WORK_BYTES)
    return fail(NEDNER_E_WORKSPACE, "workspace smaller than nedner_metrics_workspace_size");
  const double count = double(r1 - r0) * double(c1 - c0);
  const double scale = mean ? (count > 0.0 ? 1.0 / count : 0.0) : 1.0;
  const hipError_t e = nedner::launch_tenenbaum(d_img, long(rows), long(cols), long(r0), long(r1), long(c0),
                                                long(c1), dtype == NEDNER_DTYPE_F64, scale, d_result, d_work,
                                                static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NEDNER_OK : fail(NEDNER_E_HIP, std::string("tenenbaum: ") + hipGetErrorString(e));
}
}  // namespace

extern "C" {

void nedner_desc_init(nedner_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->c = 1.0;
  d->dt = 1.0;
  d->d1 = 1.0;
  d->d2 = 1.0;
  d->prec = NEDNER_FP32;
  d->w = 12;
  d->sigma = 2.0;
  d->tau_scale = 1.0;
}

nedner_status nedner_validate(const nedner_desc* desc) { return validate_impl(desc, nullptr); }

nedner_status nedner_query(const nedner_desc* desc, nedner_info* info) {
  if (!info) return fail(NEDNER_E_ARG, "info is NULL");
  Derived v;
  nedner_status st = validate_impl(desc, &v);
  if (st != NEDNER_OK) return st;
  Geometry G;
  try {
    build_geometry(*desc, v, G);
  } catch (const std::bad_alloc&) {
    return fail(NEDNER_E_OOM, "host allocation failed");
  }
  fill_info(*desc, v, int64_t(G.ent_m.size()), int64_t(G.segd.size() / 4), int64_t(G.cellbeg.size()), info);
  return NEDNER_OK;
}

nedner_status nedner_plan_create(const nedner_desc* desc, int device, void* stream, nedner_plan* plan) {
  (void)stream;
  if (!plan) return fail(NEDNER_E_ARG, "plan output pointer is NULL");
  *plan = nullptr;
  return create_one(desc, device, plan);
}

nedner_status nedner_plan_create_many(const nedner_desc* descs, int count, int device, void* stream,
                                      nedner_plan* plan) {
  (void)stream;
  if (!plan) return fail(NEDNER_E_ARG, "plan output pointer is NULL");
  *plan = nullptr;
  return create_batch(descs, count, device, plan);
}

nedner_status nedner_plan_info(nedner_plan plan, nedner_info* info) {
  if (!plan || !info) return fail(NEDNER_E_ARG, "NULL argument");
  *info = plan->info;
  return NEDNER_OK;
}

nedner_status nedner_workspace_size(nedner_plan plan, size_t* bytes) {
  if (!plan || !bytes) return fail(NEDNER_E_ARG, "NULL argument");
  *bytes = plan->need_ws;
  return NEDNER_OK;
}

nedner_status nedner_set_workspace(nedner_plan plan, void* d_ws, size_t bytes) {
  if (!plan) return fail(NEDNER_E_ARG, "plan is NULL");
  if (d_ws && (reinterpret_cast<uintptr_t>(d_ws) % 256))
    return fail(NEDNER_E_ARG, "workspace must be 256-byte aligned");
  if (d_ws && bytes < plan->need_ws)
    return fail(NEDNER_E_WORKSPACE, "workspace of " + std::to_string(bytes) + " bytes is smaller than " +
                                        std::to_string(plan->need_ws));
  plan->ws = d_ws;
  plan->ws_bytes = d_ws ? bytes : 0;
  if (!plan->subs.empty() && d_ws) return batch_upload_table(plan);
  return NEDNER_OK;
}

nedner_status nedner_execute(nedner_plan plan, const void* d_g, void* d_out, int kind, void* stream) {
  nedner_status st = exec_check(plan, kind, false);
  if (st != NEDNER_OK) return st;
  if (!d_g || !d_out) return fail(NEDNER_E_ARG, "NULL device pointer");
  DeviceGuard guard(plan->device);
  if (!guard.ok()) return fail(NEDNER_E_HIP, "cannot select the plan's device");
  return forward_impl(plan, d_g, d_out, kind, static_cast<hipStream_t>(stream));
}

nedner_status nedner_execute_adjoint(nedner_plan plan, const void* d_in, int kind, void* d_g, void* stream) {
  nedner_status st = exec_check(plan, kind, true);
  if (st != NEDNER_OK) return st;
  if (!d_in || !d_g) return fail(NEDNER_E_ARG, "NULL device pointer");
  DeviceGuard guard(plan->device);
  if (!guard.ok()) return fail(NEDNER_E_HIP, "cannot select the plan's device");
  return adjoint_impl(plan, d_in, kind, d_g, static_cast<hipStream_t>(stream));
}

nedner_status nedner_execute_q(nedner_plan plan, const void* d_v, void* d_g, void* stream) {
  nedner_status st = exec_check(plan, NEDNER_VOLUME_REAL, true);
  if (st != NEDNER_OK) return st;
  if (!d_v || !d_g) return fail(NEDNER_E_ARG, "NULL device pointer");
  DeviceGuard guard(plan->device);
  if (!guard.ok()) return fail(NEDNER_E_HIP, "cannot select the plan's device");
  const KP k = trace_params(plan);
  return adjoint_impl(plan, d_v, NEDNER_VOLUME_REAL, d_g, static_cast<hipStream_t>(stream), &k);
}

nedner_status nedner_execute_q_adjoint(nedner_plan plan, const void* d_g, void* d_v, void* stream) {
  nedner_status st = exec_check(plan, NEDNER_VOLUME_REAL, false);
  if (st != NEDNER_OK) return st;
  if (!d_g || !d_v) return fail(NEDNER_E_ARG, "NULL device pointer");
  DeviceGuard guard(plan->device);
  if (!guard.ok()) return fail(NEDNER_E_HIP, "cannot select the plan's device");
  const KP k = trace_params(plan);
  return forward_impl(plan, d_g, d_v, NEDNER_VOLUME_REAL, static_cast<hipStream_t>(stream), &k);
}

nedner_status nedner_execute_many(nedner_plan plan, const void* const* d_g, void* const* d_out, int kind,
                                  void* stream) {
  if (!plan) return fail(NEDNER_E_ARG, "plan is NULL");
  if (plan->subs.empty()) return fail(NEDNER_E_ARG, "not a batched plan: use nedner_execute");
  if (plan->broken) return fail(NEDNER_E_STATE, "plan is unusable after an earlier HIP error");
  if (kind != NEDNER_VOLUME_REAL) return fail(NEDNER_E_UNSUPPORTED, "batched execution produces volumes only");
  if (!d_g || !d_out) return fail(NEDNER_E_ARG, "NULL pointer array");
  if (!plan->ws || plan->ws_bytes < plan->need_ws)
    return fail(NEDNER_E_WORKSPACE, "no workspace, or one smaller than nedner_workspace_size");
  DeviceGuard guard(plan->device);
  if (!guard.ok()) return fail(NEDNER_E_HIP, "cannot select the plan's device");
  return execute_many_impl(plan, d_g, d_out, static_cast<hipStream_t>(stream));
}

nedner_status nedner_profile_begin(nedner_plan plan, int max_runs) {
  if (!plan) return fail(NEDNER_E_ARG, "plan is NULL");
  if (plan->broken) return fail(NEDNER_E_STATE, "plan is unusable after an earlier HIP error");
  if (max_runs < 1 || max_runs > 100000) return fail(NEDNER_E_ARG, "max_runs must be in [1, 100000]");
  DeviceGuard guard(plan->device);
  if (!guard.ok()) return fail(NEDNER_E_HIP, "cannot select the plan's device");
  free_events(plan);
  const size_t n = (size_t)max_runs * 8;  // up to 7 stage boundaries per run
  plan->ev.resize(n);
  for (size_t i = 0; i < n; ++i) {
    hipError_t e = hipEventCreate(&plan->ev[i]);
    if (e != hipSuccess) {
      plan->ev.resize(i);
      free_events(plan);
      return fail(NEDNER_E_HIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
  }
  plan->prof_max = max_runs;
  return NEDNER_OK;
}

nedner_status nedner_profile_end(nedner_plan plan, double* ms, int max_stages, int* n_stages,
                                 const char** names) {
  if (!plan || !n_stages) return fail(NEDNER_E_ARG, "NULL argument");
  DeviceGuard guard(plan->device);
  const int runs = plan->prof_runs, st = plan->prof_stages;
  *n_stages = runs > 0 ? st : 0;
  if (names) *names = runs > 0 ? plan->prof_names : "";
  std::vector<double> acc(st, 0.0);
  for (int r = 0; r < runs; ++r) {
    hipEvent_t* e = &plan->ev[(size_t)r * (st + 1)];
    hipError_t err = hipEventSynchronize(e[st]);
    if (err != hipSuccess) {
      free_events(plan);
      return fail(NEDNER_E_HIP, std::string("hipEventSynchronize: ") + hipGetErrorString(err));
    }
    for (int i = 0; i < st; ++i) {
      float t = 0.f;
      err = hipEventElapsedTime(&t, e[i], e[i + 1]);
      if (err != hipSuccess) {
        free_events(plan);
        return fail(NEDNER_E_HIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(err));
      }
      acc[i] += t;
    }
  }
  if (ms)
    for (int i = 0; i < st && i < max_stages; ++i) ms[i] = runs ? acc[i] / runs : 0.0;
  free_events(plan);
  return NEDNER_OK;
}

nedner_status nedner_get_tuning(nedner_plan plan, nedner_tuning* t) {
  if (!plan || !t) return fail(NEDNER_E_ARG, "NULL argument");
  get_tuning(plan->subs.empty() ? plan : plan->subs[0], t);
  return NEDNER_OK;
}

nedner_status nedner_set_tuning(nedner_plan plan, const nedner_tuning* t) {
  if (!plan || !t) return fail(NEDNER_E_ARG, "NULL argument");
  if (!plan->subs.empty()) return fail(NEDNER_E_UNSUPPORTED, "set_tuning applies to single-problem plans");
  if (plan->broken) return fail(NEDNER_E_STATE, "plan is unusable after an earlier HIP error");
  if (!pass_shape_ok(t->pass_lines, t->pass_threads) || t->spread_depth != 1 ||
      t->rows_per_wave < 1 || t->gather_rows < 0)
    return fail(NEDNER_E_ARG, "invalid tuning");
  if (t->gather_rows > 0 && !sweep_gather_ok(plan->kp))
    return fail(NEDNER_E_ARG, "the sweep gather takes float plans with w <= 12");
  nedner_status st = set_spread_shape(plan, t->rows_per_wave, t->time_per_lane, t->spread_depth);
  if (st != NEDNER_OK) return st;
  plan->kp.pass_lines = t->pass_lines;
  plan->kp.pass_threads = t->pass_threads;
  plan->kp.pass_ip = t->pass_inplace != 0;
  plan->kp.gS = t->gather_rows;
  return NEDNER_OK;
}

nedner_status nedner_autotune(nedner_plan plan, const void* d_g, void* stream, nedner_tuning* best) {
  if (!plan) return fail(NEDNER_E_ARG, "plan is NULL");
  if (plan->broken) return fail(NEDNER_E_STATE, "plan is unusable after an earlier HIP error");
  DeviceGuard guard(plan->device);
  if (!guard.ok()) return fail(NEDNER_E_HIP, "cannot select the plan's device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return plan->subs.empty() ? autotune_single(plan, d_g, s, best) : autotune_batch(plan, s, best);
}

size_t nedner_metrics_workspace_size(void) { return nedner::METRICS_WORK_BYTES; }

nedner_status nedner_mip(const void* d_vol, int n1, int n2, int n3, int axis, int dtype, void* d_out,
                         void* stream) {
  if (!d_vol || !d_out) return fail(NEDNER_E_ARG, "NULL device pointer");
  if (n1 < 1 || n2 < 1 || n3 < 1) return fail(NEDNER_E_ARG, "volume sizes must be positive");
  if (axis < 0 || axis > 2) return fail(NEDNER_E_ARG, "axis must be 0, 1 or 2");
  if (dtype != NEDNER_DTYPE_F32 && dtype != NEDNER_DTYPE_F64) return fail(NEDNER_E_ARG, "unknown dtype");
  const hipError_t e = nedner::launch_mip(d_vol, n1, n2, n3, axis, dtype == NEDNER_DTYPE_F64, d_out,
                                          static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NEDNER_OK : fail(NEDNER_E_HIP, std::string("mip: ") + hipGetErrorString(e));
}

nedner_status nedner_corrcoef(const void* d_a, const void* d_b, const unsigned char* d_mask, int64_t n,
                              int dtype, double* d_result, void* d_work, size_t work_bytes, void* stream) {
  if (!d_a || !d_b || !d_result || !d_work) return fail(NEDNER_E_ARG, "NULL device pointer");
  if (n < 1) return fail(NEDNER_E_ARG, "n must be positive");
  if (dtype != NEDNER_DTYPE_F32 && dtype != NEDNER_DTYPE_F64) return fail(NEDNER_E_ARG, "unknown dtype");
  if (work_bytes < nedner::METRICS_WORK_BYTES)
    return fail(NEDNER_E_WORKSPACE, "workspace smaller than nedner_metrics_workspace_size");
  const hipError_t e = nedner::launch_corrcoef(d_a, d_b, d_mask, long(n), dtype == NEDNER_DTYPE_F64, d_result,
                                               d_work, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NEDNER_OK : fail(NEDNER_E_HIP, std::string("corrcoef: ") + hipGetErrorString(e));
}


nedner_status nedner_corrcoef_noalloc(const void* d_a, const void* d_b, const unsigned char* d_mask, int64_t n,
                                      int dtype, double* d_result, void* stream) {
  if (!d_a || !d_b || !d_result) return fail(NEDNER_E_ARG, "NULL device pointer");
  if (n < 1) return fail(NEDNER_E_ARG, "n must be positive");
  if (dtype != NEDNER_DTYPE_F32 && dtype != NEDNER_DTYPE_F64) return fail(NEDNER_E_ARG, "unknown dtype");
  // the scratch holds a fixed number of partial sums whatever n: there is no
  // input size it cannot serve
  if (nedner::noalloc_scratch_bytes() > nedner::METRICS_WORK_BYTES)
    return fail(NEDNER_E_WORKSPACE, "scratch larger than its stated maximum");
  const hipError_t e = nedner::launch_corrcoef_noalloc(d_a, d_b, d_mask, long(n), dtype == NEDNER_DTYPE_F64,
                                                       d_result, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? NEDNER_OK
                         : fail(NEDNER_E_HIP, std::string("corrcoef_noalloc: ") + hipGetErrorString(e));
}

nedner_status nedner_tenenbaum(const void* d_img, int64_t rows, int64_t cols, int64_t r0, int64_t r1,
                               int64_t c0, int64_t c1, int dtype, double* d_result, void* d_work,
                               size_t work_bytes, void* stream) {
  return tenenbaum_impl(d_img, rows, cols, r0, r1, c0, c1, dtype, false, d_result, d_work, work_bytes, stream);
}

nedner_status nedner_tenenbaum_mean(const void* d_img, int64_t rows, int64_t cols, int64_t r0, int64_t r1,
                                    int64_t c0, int64_t c1, int dtype, double* d_result, void* d_work,
                                    size_t work_bytes, void* stream) {
  return tenenbaum_impl(d_img, rows, cols, r0, r1, c0, c1, dtype, true, d_result, d_work, work_bytes, stream);
}

nedner_status nedner_debug_inject_hip_error(nedner_plan plan, int code) {
  if (!plan) return fail(NEDNER_E_ARG, "plan is NULL");
  if (code == int(hipSuccess)) return fail(NEDNER_E_ARG, "an injected error code must not be hipSuccess");
  for (nedner_plan sp : plan->subs) sp->broken = true;
  return hip_fail(plan, static_cast<hipError_t>(code), "injected by nedner_debug_inject_hip_error");
}

nedner_status nedner_destroy(nedner_plan plan) {
  destroy_one(plan);
  return NEDNER_OK;
}

const char* nedner_status_string(nedner_status s) {
  switch (s) {
    case NEDNER_OK: return "ok";
    case NEDNER_E_ARG: return "invalid argument";
    case NEDNER_E_ALIAS: return "time sampling aliases";
    case NEDNER_E_OOM: return "out of memory";
    case NEDNER_E_WORKSPACE: return "workspace missing or too small";
    case NEDNER_E_HIP: return "HIP runtime error";
    case NEDNER_E_UNSUPPORTED: return "unsupported";
    case NEDNER_E_STATE: return "plan unusable";
  }
  return "unknown status";
}

const char* nedner_last_error(void) { return g_last_error.c_str(); }

int nedner_version(void) { return NEDNER_VERSION; }

}  // extern "C"

// Host checks of the library's validation and plan geometry under
// AddressSanitizer and UndefinedBehaviorSanitizer: nedner_validate and
// nedner_query (which builds the sensor cells, window tables and spreading
// lists) on seeded descriptors, valid and invalid: sensors on the aperture's
// edges and corners, wrapped positions, one sensor, many sensors in one cell,
// sweep lengths from 1 to the whole grid, every precision and window, the
// two-dimensional and equispaced cases, and arguments out of range. A memory
// error or undefined behaviour aborts the program; otherwise it prints the
// number of descriptors checked and exits 0.
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <random>
#include <vector>

#include "nedner.h"

namespace {

int g_checked = 0;

nedner_status run(nedner_desc d) {
  const nedner_status a = nedner_validate(&d);
  nedner_info info;
  const nedner_status b = nedner_query(&d, &info);
  if (a != b && !(a == NEDNER_OK && b == NEDNER_E_OOM)) {
    std::fprintf(stderr, "validate %d and query %d disagree\n", int(a), int(b));
    std::abort();
  }
  if (b == NEDNER_OK && (info.list_entries < 0 || info.workspace_bytes == 0)) {
    std::fprintf(stderr, "implausible query result\n");
    std::abort();
  }
  if (nedner_last_error() == nullptr || nedner_status_string(b) == nullptr) std::abort();
  ++g_checked;
  return b;
}

}  // namespace

int main() {
  std::mt19937_64 rng(20150112);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  const int precs[] = {NEDNER_FP64, NEDNER_FP32, NEDNER_FP32_COMPENSATED, NEDNER_FP32_PLAIN, NEDNER_FP32_WIDE};
  for (int iter = 0; iter < 400; ++iter) {
    nedner_desc d;
    nedner_desc_init(&d);
    const int layout = iter % 8;
    int64_t m = 1 + int64_t(rng() % 600);
    if (layout == 3) m = 1;
    std::vector<double> xy(2 * size_t(m)), h(size_t(m), 1.0 / double(m));
    for (int64_t i = 0; i < m; ++i) {
      double x = U(rng), y = U(rng);
      if (layout == 1) x = (i % 2) ? 0.0 : std::nextafter(1.0, 0.0);  // aperture edges
      if (layout == 2) x = y = 0.5;                                      // one cell
      if (layout == 4) y = 0.0;                                           // one row
      xy[2 * i] = x;
      xy[2 * i + 1] = y;
    }
    d.m = m;
    d.xy = xy.data();
    d.h = (iter % 3) ? h.data() : nullptr;
    const int sizes[] = {2, 4, 6, 8, 10, 12, 16, 20, 24, 30, 32, 40, 48};
    d.n1 = sizes[rng() % 13];
    d.n2 = layout == 5 ? 1 : sizes[rng() % 13];
    d.n3 = sizes[rng() % 13];
    d.nt = 2 * (1 + int64_t(rng() % 64));
    d.dt = 1.0 / double(d.nt);
    d.c = 0.5 + U(rng);
    d.t0 = (iter % 5 == 0) ? 0.01 : 0.0;
    d.d1 = 1.0 / d.n1;
    d.d2 = 1.0 / d.n2;
    d.prec = precs[iter % 5];
    d.w = 2 * (1 + int(rng() % 8));
    d.window = (iter % 7 == 0) ? NEDNER_WINDOW_KAISER_BESSEL : NEDNER_WINDOW_GAUSSIAN;
    d.rows_per_wave = int(rng() % 3) == 0 ? 0 : 1 + int(rng() % 64);
    d.time_per_lane = int(rng() % 4) == 3 ? 4 : int(rng() % 3);
    d.flags = NEDNER_ALLOW_ALIAS | ((layout == 6) ? NEDNER_WRAP_POSITIONS : 0u);
    if (layout == 6)
      for (auto& v : xy) v = 3.0 * v - 1.0;  // outside the aperture: wrapped
    if (layout == 7) {
      // sensors on the output grid's nodes
      d.flags |= NEDNER_EQUISPACED;
      for (int64_t i = 0; i < m; ++i) {
        xy[2 * i] = double(i % d.n1) * d.d1;
        xy[2 * i + 1] = double((i / d.n1) % (d.n2 > 1 ? d.n2 : 1)) * d.d2;
      }
    }
    run(d);
    // the same descriptor with one argument out of range
    nedner_desc bad = d;
    switch (iter % 6) {
      case 0: bad.nt = 3; break;
      case 1: bad.w = 17; break;
      case 2: bad.dt = -1.0; break;
      case 3: bad.n1 = 7; break;
      case 4: bad.prec = 9; break;
      default: bad.flags = d.flags & ~NEDNER_WRAP_POSITIONS; xy[0] = 2.0; break;
    }
    if (run(bad) == NEDNER_OK && iter % 6 != 5) {
      std::fprintf(stderr, "an invalid descriptor was accepted (case %d)\n", iter % 6);
      return 1;
    }
  }
  if (nedner_validate(nullptr) != NEDNER_E_ARG) return 1;
  std::printf("checked %d descriptors\n", g_checked);
  return 0;
}

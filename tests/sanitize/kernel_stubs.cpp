// Stand-ins for the kernel launchers of the library, so that its host part
// (descriptor validation and the plan geometry: sensor cells, window tables,
// spreading lists) links into an AddressSanitizer / UndefinedBehaviorSanitizer
// build without device code. The checks never reach a launch; each stand-in
// reports that it is not available.
#include "batch.hpp"

namespace nedner {

namespace {
hipError_t unavailable() { return hipErrorNotSupported; }
}  // namespace

hipError_t launch_spread(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_place(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_place_adj(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
int spread_blocks_per_cu(const KP&) { return 1; }
hipError_t launch_mip(const void*, int, int, int, int, bool, void*, hipStream_t) { return unavailable(); }
hipError_t launch_corrcoef(const void*, const void*, const unsigned char*, long, bool, double*, void*,
                           hipStream_t) {
  return unavailable();
}
hipError_t launch_tenenbaum(const void*, long, long, long, long, long, long, bool, double, double*, void*,
                            hipStream_t) {
  return unavailable();
}
hipError_t launch_corrcoef_noalloc(const void*, const void*, const unsigned char*, long, bool, double*,
                                   hipStream_t) {
  return unavailable();
}
size_t noalloc_scratch_bytes() { return 0; }
hipError_t launch_gather(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_lat_a(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_lat_b(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_column(const KP&, const void*, void*, int, hipStream_t) { return unavailable(); }
hipError_t launch_pass_c(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_pass_d(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_adj_d(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_adj_c(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_column_adj(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_adj_b(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_adj_a(const KP&, const void*, void*, hipStream_t) { return unavailable(); }
hipError_t launch_batch_prepare(BatchProb*, const PtrChunk&, int*, int, hipStream_t) { return unavailable(); }
hipError_t launch_spread_many(const KP&, const BatchProb*, const WorkList&, int, hipStream_t) {
  return unavailable();
}
hipError_t launch_pass_many(const KP&, int, const BatchProb*, const WorkList&, size_t, hipStream_t) {
  return unavailable();
}
hipError_t launch_column_many(const KP&, const BatchProb*, const WorkList&, int, size_t, hipStream_t) {
  return unavailable();
}
size_t column_wave_bytes_host(const KP&) { return 0; }
int column_wpc_host(const KP&) { return 1; }
int column_ppt_host(const KP&) { return 4; }
size_t column_shared_bytes_host(const KP&) { return 0; }

}  // namespace nedner

// Host-side dispatch of the NER column kernels (k_column_impl.hpp) over the
// precisions, each of which is compiled in a translation unit of its own.
#include "k_column_impl.hpp"

namespace nedner {

extern template hipError_t column_a<double, true>(const KP&, const void*, void*, int, hipStream_t, bool);
extern template hipError_t column_many_a<double, true>(const KP&, int, const BatchProb*, const WorkList&, int, size_t,
                                                   hipStream_t);
extern template hipError_t column_a<float, true>(const KP&, const void*, void*, int, hipStream_t, bool);
extern template hipError_t column_many_a<float, true>(const KP&, int, const BatchProb*, const WorkList&, int, size_t,
                                                   hipStream_t);
extern template hipError_t column_a<float, false>(const KP&, const void*, void*, int, hipStream_t, bool);
extern template hipError_t column_many_a<float, false>(const KP&, int, const BatchProb*, const WorkList&, int, size_t,
                                                   hipStream_t);

static hipError_t column_dispatch(const KP& p, const void* in, void* out, int spec, hipStream_t s, bool adj) {
  switch (p.prec) {
    case PREC_FP64: return column_a<double, true>(p, in, out, spec, s, adj);
    case PREC_FP32P: return column_a<float, false>(p, in, out, spec, s, adj);
    default: return column_a<float, true>(p, in, out, spec, s, adj);
  }
}

// cpw columns per workgroup and `smem` bytes of LDS (the maxima over the batch);
// the register bound follows the largest per-column transform in p0.
hipError_t launch_column_many(const KP& p0, const BatchProb* bp, const WorkList& wl, int cpw, size_t smem,
                              hipStream_t s) {
  const int ppt = column_ppt(p0);
  switch (p0.prec) {
    case PREC_FP64: return column_many_a<double, true>(p0, ppt, bp, wl, cpw, smem, s);
    case PREC_FP32P: return column_many_a<float, false>(p0, ppt, bp, wl, cpw, smem, s);
    default: return column_many_a<float, true>(p0, ppt, bp, wl, cpw, smem, s);
  }
}

// host helpers for the batched plan: LDS of one column and of the shared
// twiddles, wavefronts per column
int column_wpc_host(const KP& p) { return column_wpc(p.ntt, p.N3); }
int column_ppt_host(const KP& p) { return column_ppt(p); }
size_t column_wave_bytes_host(const KP& p) {
  return p.prec == PREC_FP64 ? col_wave_bytes<double>(p.ntt, p.N3, false)
                             : col_wave_bytes<float>(p.ntt, p.N3, false);
}
size_t column_shared_bytes_host(const KP& p) {
  return p.prec == PREC_FP64 ? col_shared_bytes<double>(p.ntt, p.N3) : col_shared_bytes<float>(p.ntt, p.N3);
}

hipError_t launch_column(const KP& p, const void* G, void* out, int spectrum, hipStream_t s) {
  return column_dispatch(p, G, out, spectrum, s, false);
}

hipError_t launch_column_adj(const KP& p, const void* Z1, void* G, hipStream_t s) {
  return column_dispatch(p, Z1, G, 0, s, true);
}

}  // namespace nedner

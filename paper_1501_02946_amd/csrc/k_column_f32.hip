// NER column kernels instantiated for FP32 data with FP64 frequency and phase arguments (fp32, fp32c, fp32w).
#include "k_column_impl.hpp"

namespace nedner {

template hipError_t column_a<float, true>(const KP&, const void*, void*, int, hipStream_t, bool);
template hipError_t column_many_a<float, true>(const KP&, int, const BatchProb*, const WorkList&, int, size_t,
                                            hipStream_t);

}  // namespace nedner

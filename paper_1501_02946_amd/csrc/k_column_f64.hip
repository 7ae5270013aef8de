// NER column kernels instantiated for FP64.
#include "k_column_impl.hpp"

namespace nedner {

template hipError_t column_a<double, true>(const KP&, const void*, void*, int, hipStream_t, bool);
template hipError_t column_many_a<double, true>(const KP&, int, const BatchProb*, const WorkList&, int, size_t,
                                            hipStream_t);

}  // namespace nedner

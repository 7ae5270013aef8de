// Spreading and sensor-gather kernels instantiated for FP32 and FP32 plain (float data, weights and sums).
#include "k_spread_impl.hpp"

namespace nedner {

template hipError_t spread_p<float, float, float, false>(const KP&, const void*, void*, int, hipStream_t, bool);
template hipError_t spread_many_p<float, float, float, false>(const KP&, const BatchProb*, const WorkList&, bool,
                                                      hipStream_t);
template int occ_p<float, float, float, false>(const KP&);

}  // namespace nedner

// Spreading and sensor-gather kernels instantiated for compensated FP32
// (float data and weights, Kahan-compensated float sums).
#include "k_spread_impl.hpp"

namespace nedner {

template hipError_t spread_p<float, float, float, true>(const KP&, const void*, void*, int, hipStream_t, bool);
template hipError_t spread_many_p<float, float, float, true>(const KP&, const BatchProb*, const WorkList&, bool,
                                                      hipStream_t);
template int occ_p<float, float, float, true>(const KP&);

}  // namespace nedner

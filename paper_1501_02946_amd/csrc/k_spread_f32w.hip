// Spreading and sensor-gather kernels instantiated for FP32 with wide sums
// (float data, double sums; double or float first-axis weights).
#include "k_spread_impl.hpp"

namespace nedner {

template hipError_t spread_p<float, double, double, false>(const KP&, const void*, void*, int, hipStream_t, bool);
template hipError_t spread_many_p<float, double, double, false>(const KP&, const BatchProb*, const WorkList&, bool,
                                                      hipStream_t);
template int occ_p<float, double, double, false>(const KP&);
template hipError_t spread_p<float, float, double, false>(const KP&, const void*, void*, int, hipStream_t, bool);
template hipError_t spread_many_p<float, float, double, false>(const KP&, const BatchProb*, const WorkList&, bool,
                                                      hipStream_t);
template int occ_p<float, float, double, false>(const KP&);

}  // namespace nedner

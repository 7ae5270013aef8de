// Spreading and sensor-gather kernels instantiated for FP64 (double data, weights and sums).
#include "k_spread_impl.hpp"

namespace nedner {

template hipError_t spread_p<double, double, double, false>(const KP&, const void*, void*, int, hipStream_t, bool);
template hipError_t spread_many_p<double, double, double, false>(const KP&, const BatchProb*, const WorkList&, bool,
                                                      hipStream_t);
template int occ_p<double, double, double, false>(const KP&);

}  // namespace nedner

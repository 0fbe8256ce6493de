// Instantiation of the solver kernels and launch sequence for padded block size 12.
#include "launch_impl.hpp"

namespace rcr {
template int launch_all_m<double, 12>(PlanObj &, Bufs<double>, Timer &, hipStream_t);
}  // namespace rcr

// Instantiation of the solver kernels and launch sequence for padded block size 4.
#include "launch_impl.hpp"

namespace rcr {
template int launch_all_m<double, 4>(PlanObj &, Bufs<double>, Timer &, hipStream_t);
}  // namespace rcr

// Instantiation of the solver kernels and launch sequences for padded block size 6.
#include "launch_impl.hpp"

namespace rcr {
template int launch_phase_m<double, 6>(PlanObj &, Bufs<double>, Timer &, hipStream_t, int);
template int launch_phase_m<float, 6>(PlanObj &, Bufs<float>, Timer &, hipStream_t, int);
}  // namespace rcr

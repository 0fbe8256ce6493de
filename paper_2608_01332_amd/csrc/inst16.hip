// Instantiation of the solver kernels and launch sequences for padded block size 16.
#include "launch_impl.hpp"

namespace rcr {
template int launch_phase_m<double, 16>(PlanObj &, Bufs<double>, Timer &, hipStream_t, int);
template int launch_phase_m<float, 16>(PlanObj &, Bufs<float>, Timer &, hipStream_t, int);
}  // namespace rcr

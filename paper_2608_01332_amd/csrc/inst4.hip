// Instantiation of the solver kernels and launch sequences for padded block size 4.
#include "launch_impl.hpp"

namespace rcr {
template int launch_phase_m<double, 4>(PlanObj &, Bufs<double>, Timer &, hipStream_t, int);
template int launch_phase_m<float, 4>(PlanObj &, Bufs<float>, Timer &, hipStream_t, int);
}  // namespace rcr

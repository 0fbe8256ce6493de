// Instantiation of the solver kernels and launch sequences for padded block size 8.
#include "launch_impl.hpp"

namespace rcr {
template int launch_phase_m<double, 8>(PlanObj &, Bufs<double>, Timer &, hipStream_t, int);
template int launch_phase_m<float, 8>(PlanObj &, Bufs<float>, Timer &, hipStream_t, int);
}  // namespace rcr

// Instantiation of the solver kernels and launch sequences for padded block size 12.
#include "launch_impl.hpp"

namespace rcr {
template int launch_phase_m<double, 12>(PlanObj &, Bufs<double>, Timer &, hipStream_t, int);
template int launch_phase_m<float, 12>(PlanObj &, Bufs<float>, Timer &, hipStream_t, int);
}  // namespace rcr

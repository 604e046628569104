// Double-precision instantiation of the step kernels. Built with
// -ffp-contract=off: every FP64 expression rounds exactly as the CPU oracle's.
#include "mhd_kernels_impl.h"

namespace mhd {
template hipError_t launch_cfl<double>(const double*, const double*, Grid, double, double, Ctl*, hipStream_t);
template hipError_t launch_cmax_only<double>(const double*, const double*, Grid, double, Ctl*, hipStream_t);
template hipError_t launch_divb<double>(const double*, Grid, Ctl*, hipStream_t);
template hipError_t launch_fluid<double>(int, const double*, double*, const double*, Grid, double, const Ctl*,
                                         double, hipStream_t);
template hipError_t launch_ct<double>(int, const double*, const double*, double*, Grid, const Ctl*, double,
                                      hipStream_t);
}  // namespace mhd

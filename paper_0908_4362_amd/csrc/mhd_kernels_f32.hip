// Single-precision instantiation of the step kernels (FMA contraction allowed).
#include "mhd_kernels_impl.h"

namespace mhd {
template hipError_t launch_cfl<float>(const float*, const float*, Grid, double, unsigned long long*, int*,
                                      hipStream_t);
template hipError_t launch_divb<float>(const float*, Grid, unsigned long long*, int*, hipStream_t);
template hipError_t launch_fluid<float>(int, const float*, float*, const float*, Grid, double, const Ctl*, double,
                                        unsigned long long*, int*, hipStream_t);
template hipError_t launch_ct<float>(int, const float*, const float*, float*, Grid, const Ctl*, double,
                                     hipStream_t);
}  // namespace mhd

// Single-precision instantiation of the step kernels. Built with
// -ffp-contract=on: a multiply and an add fuse into an FMA only within one
// source expression, never across statements, so results do not depend on
// where a loop's unrolled copies place an iteration (chunk layout, tiles).
#include "mhd_batch_impl.h"
#include "mhd_diag_impl.h"
#include "mhd_flat_impl.h"

namespace mhd {
template hipError_t launch_cfl<float>(const float*, const float*, Grid, double, unsigned long long*, Ctl*,
                                      hipStream_t);
template hipError_t launch_divb<float>(const float*, Grid, unsigned long long*, int*, hipStream_t);
template hipError_t launch_fluid<float>(int, const float*, float*, const float*, Grid, double, Ctl*, double,
                                        unsigned long long*, hipStream_t);
template hipError_t launch_ct<float>(int, const float*, const float*, float*, Grid, const Ctl*, double,
                                     hipStream_t);
template hipError_t launch_ct_flat<float>(int, const float*, const float*, float*, Grid, const Ctl*, double,
                                           hipStream_t);
template hipError_t launch_ct_fluid<float>(int, const float*, float*, const float*, float*, Grid, double, Ctl*, double,
                                           unsigned long long*, hipStream_t);
template bool fused_reverse_pays<float>(const Grid&, int);
template void tile_default<float>(const Grid&, int, int*, int*);
template void tile_candidates<float>(const Grid&, int, std::vector<std::pair<int, int>>&);
template unsigned tile_blocks<float>(const Grid&, int, int, int);
template hipError_t launch_batch<float>(int, bool, const BJob*, const TileDesc*, int, unsigned, int, int,
                                         hipStream_t, long long);
template hipError_t launch_diag<float>(const float*, const float*, Grid, double, int, int, int, float*, hipStream_t);
template hipError_t launch_validate<float>(const float*, const float*, long long, Ctl*, hipStream_t);
}  // namespace mhd

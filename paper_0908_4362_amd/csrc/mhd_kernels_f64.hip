// Double-precision instantiation of the step kernels, plus the
// precision-independent launchers. Built with -ffp-contract=off: every FP64
// expression rounds exactly as the CPU oracle's.
#include "mhd_batch_impl.h"
#include "mhd_diag_impl.h"
#include "mhd_flat_impl.h"

namespace mhd {
namespace {
// Second level of a grid-wide max: one block reduces the per-block maxima;
// what = 0: the ctl->nparts slots of the last c_max producer into ctl->cmax,
// then (cfl > 0) the time-step rule; what = 1: nparts slots of max |div B|
// into ctl->divb.
constexpr int FB = 1024;   // threads of the finisher
__global__ void __launch_bounds__(FB) finish_kernel(const unsigned long long* __restrict__ parts, int nparts,
                                                    int what, double cfl, Ctl* ctl)
{
    if (what == 0) nparts = ctl->nparts;
    unsigned long long best = 0ull;
    // unrolled so that each thread has several loads in flight (up to 80
    // slots per thread when an x sweep produced them)
#pragma unroll 8
    for (int k = threadIdx.x; k < nparts; k += FB) best = parts[k] > best ? parts[k] : best;
    best = block_max_u64<FB>(best, threadIdx.x);
    if (threadIdx.x == 0) {
        const double m = __longlong_as_double((long long)best);
        if (what == 1) {
            ctl->divb = m;
        } else {
            ctl->cmax = m;
            if (cfl > 0.0) apply_dt_rule(ctl, cfl);
        }
    }
}

// Batched second level: workgroup j reduces the maxima of problem j (as many
// as the producing launch gave it workgroups) and applies its dt rule.
constexpr int FBB = 256;
__global__ void __launch_bounds__(FBB) finish_batch_kernel(const BJob* __restrict__ jobs,
                                                           const TileDesc* __restrict__ td, double cfl)
{
    const int j = blockIdx.x;
    const unsigned long long* parts = jobs[j].parts;
    const unsigned n = td[j + 1].first - td[j].first;
    unsigned long long best = 0ull;
#pragma unroll 8
    for (unsigned k = threadIdx.x; k < n; k += FBB) best = parts[k] > best ? parts[k] : best;
    best = block_max_u64<FBB>(best, threadIdx.x);
    if (threadIdx.x == 0) {
        Ctl* ctl = jobs[j].ctl;
        ctl->cmax = __longlong_as_double((long long)best);
        if (cfl > 0.0) apply_dt_rule(ctl, cfl);
    }
}

}  // namespace

hipError_t launch_finish_batch(const BJob* jobs, const TileDesc* td, int njobs, double cfl, hipStream_t s)
{
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(finish_batch_kernel, dim3(njobs), dim3(FBB), 0, s, jobs, td, cfl);
    return hipGetLastError();
}

hipError_t launch_finish(const unsigned long long* parts, int nparts, int what, double cfl, Ctl* ctl, hipStream_t s)
{
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(FB), 0, s, parts, nparts, what, cfl, ctl);
    return hipGetLastError();
}

int reduce_slots(const Grid& g) { return reduce_blocks(g); }

size_t reduce_capacity(const Grid& g)
{
    size_t cap = (size_t)reduce_blocks(g);
    cap = std::max(cap, (size_t)x_wave_blocks(g));
    cap = std::max(cap, (size_t)ct_fluid_x_blocks(g));
    cap = std::max(cap, (size_t)g.n[1] * (size_t)g.n[2]);   // row form of the fused x sweep (FP64)
    for (int axis = 1; axis <= 2; axis++) {
        cap = std::max(cap, (size_t)march_blocks(g, axis, march_chunk(g, axis, GF, kFluidMarchWaves, true), true));
        for (int c : {fused_chunk<double>(g, axis), fused_chunk<float>(g, axis)})
            for (bool xw : {true, false}) cap = std::max(cap, (size_t)march_blocks(g, axis, c, xw));
    }
    return cap;
}

template hipError_t launch_cfl<double>(const double*, const double*, Grid, double, unsigned long long*, Ctl*,
                                       hipStream_t);
template hipError_t launch_divb<double>(const double*, Grid, unsigned long long*, int*, hipStream_t);
template hipError_t launch_fluid<double>(int, const double*, double*, const double*, Grid, double, Ctl*,
                                         double, unsigned long long*, hipStream_t);
template hipError_t launch_ct<double>(int, const double*, const double*, double*, Grid, const Ctl*, double,
                                      hipStream_t);
template hipError_t launch_ct_flat<double>(int, const double*, const double*, double*, Grid, const Ctl*, double,
                                           hipStream_t);
template hipError_t launch_ct_fluid<double>(int, const double*, double*, const double*, double*, Grid, double, Ctl*, double,
                                           unsigned long long*, hipStream_t);
template bool fused_reverse_pays<double>(const Grid&, int);
template void tile_default<double>(const Grid&, int, int*, int*);
template void tile_candidates<double>(const Grid&, int, std::vector<std::pair<int, int>>&);
template unsigned tile_blocks<double>(const Grid&, int, int, int);
template hipError_t launch_batch<double>(int, bool, const BJob*, const TileDesc*, int, unsigned, int, int,
                                         hipStream_t, long long);
template hipError_t launch_diag<double>(const double*, const double*, Grid, double, int, int, int, double*, hipStream_t);
template hipError_t launch_validate<double>(const double*, const double*, long long, Ctl*, hipStream_t);
}  // namespace mhd

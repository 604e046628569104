// Batched launches of the step kernels: one launch runs one sub-operation
// (a directional fluid or field sweep, or the CFL reduction) for every
// problem of a batch, whatever their grid sizes. A workgroup finds its
// problem by binary search over the per-problem workgroup ranges, then runs
// the same kernel body as the single-problem launch with that problem's grid,
// buffers, control block and tile parameters, so every problem gets exactly
// the arithmetic of a plain solve. The cache policy of a launch's accesses
// (non-temporal stores and read-once loads, or plain ones) follows the total
// state of its problems (512 Alfven problems, 309.6 M cells FP32: 8.70 ->
// 9.02 G cell-updates/s with non-temporal stores, 9.33 -> 9.38 G with the
// loads as well).
#pragma once
#include "mhd_kernels_impl.h"

namespace mhd {
namespace {

// Problem owning logical workgroup w: the last j with td[j].first <= w.
__device__ __forceinline__ int find_job(const TileDesc* __restrict__ td, int njobs, unsigned w)
{
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (td[mid].first <= w)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

template <typename T, int D, bool CFL, bool NT>
__global__ void __launch_bounds__(64 * MW) fluid_march_batch(const BJob* __restrict__ jobs,
                                                             const TileDesc* __restrict__ td, int njobs, int iu,
                                                             int ib)
{
    const int j = find_job(td, njobs, blockIdx.x);
    const BJob& J = jobs[j];
    const Grid g = J.g;
    const unsigned lb = blockIdx.x - td[j].first;
    fluid_march_body<T, D, CFL, NT>(static_cast<const T*>(J.u[iu]), static_cast<T*>(J.u[iu ^ 1]),
                                static_cast<const T*>(J.b[ib]), g, (T)J.gamma, J.ctl, -1.0, td[j].p0, lb,
                                J.parts + lb);
}

template <typename T, int D, bool NT>
__global__ void __launch_bounds__(64 * MW) ct_march_batch(const BJob* __restrict__ jobs,
                                                          const TileDesc* __restrict__ td, int njobs, int iu, int ib)
{
    const int j = find_job(td, njobs, blockIdx.x);
    const BJob& J = jobs[j];
    const Grid g = J.g;
    const unsigned lb = blockIdx.x - td[j].first;
    ct_march_body<T, D, NT>(static_cast<const T*>(J.u[iu]), static_cast<const T*>(J.b[ib]), static_cast<T*>(J.b[ib ^ 1]),
                        g, J.ctl, -1.0, td[j].p0, lb);
}

// x sweeps: tile p0 = 0 runs the wavefront form, p0 = K with p1 = W the
// lane-row form with K cells per lane and W lanes per row (FP32 periodic rows
// of W K cells: 64, 128, 32, 96 and 48 cells).
#define MHD_BATCH_LROW_DISPATCH(K, W, X) \
    switch ((K) * 100 + (W)) {           \
    case 164: X(1, 64) break;            \
    case 264: X(2, 64) break;            \
    case 132: X(1, 32) break;            \
    case 332: X(3, 32) break;            \
    default: X(3, 16) break;             \
    }
template <typename T, bool CFL, bool NT>
__global__ void __launch_bounds__(256) fluid_x_batch(const BJob* __restrict__ jobs, const TileDesc* __restrict__ td,
                                                     int njobs, int iu, int ib)
{
    const int j = find_job(td, njobs, blockIdx.x);
    const BJob& J = jobs[j];
    const Grid g = J.g;
    const unsigned lb = blockIdx.x - td[j].first;
    const T* uin = static_cast<const T*>(J.u[iu]);
    T* uout = static_cast<T*>(J.u[iu ^ 1]);
    const T* bf = static_cast<const T*>(J.b[ib]);
    if constexpr (!kExact<T>) {
        if (td[j].p0) {
#define MHD_LROW_BFLUID(KK, WW) \
    fluid_x_lrow_body<T, KK, WW, CFL, NT>(uin, uout, bf, g, (T)J.gamma, J.ctl, -1.0, lb, J.parts + lb);
            MHD_BATCH_LROW_DISPATCH(td[j].p0, td[j].p1, MHD_LROW_BFLUID)
#undef MHD_LROW_BFLUID
            return;
        }
    }
    fluid_x_body<T, CFL, NT>(uin, uout, bf, g, (T)J.gamma, J.ctl, -1.0, lb, J.parts + lb);
}

template <typename T, bool NT>
__global__ void __launch_bounds__(256) ct_x_batch(const BJob* __restrict__ jobs, const TileDesc* __restrict__ td,
                                                  int njobs, int iu, int ib)
{
    const int j = find_job(td, njobs, blockIdx.x);
    const BJob& J = jobs[j];
    const Grid g = J.g;
    const unsigned lb = blockIdx.x - td[j].first;
    const T* uf = static_cast<const T*>(J.u[iu]);
    const T* bin = static_cast<const T*>(J.b[ib]);
    T* bout = static_cast<T*>(J.b[ib ^ 1]);
    if constexpr (!kExact<T>) {
        if (td[j].p0) {
#define MHD_LROW_BCT(KK, WW) ct_x_lrow_body<T, KK, WW, NT>(uf, bin, bout, g, J.ctl, -1.0, lb);
            MHD_BATCH_LROW_DISPATCH(td[j].p0, td[j].p1, MHD_LROW_BCT)
#undef MHD_LROW_BCT
            return;
        }
    }
    ct_x_body<T, NT>(uf, bin, bout, g, J.ctl, -1.0, lb);
}

// Lane-row cells per lane (and in *W the lanes per row) a batched x sweep may
// take for this grid (0: none): the shapes MHD_BATCH_LROW_DISPATCH covers.
template <typename T>
int batch_x_lrow_k(const Grid& g, int* W)
{
    if (kExact<T>) return 0;
    const int k = x_lrow_k(g, W, 3);
    return (k == 3 && *W == 64) ? 0 : k;
}

// Fused reverse L_d (periodic problems only; a cohort runs them only when
// every member is periodic): y/z as ct_fluid_march, x as ct_fluid_x_body or,
// with p0 = K, the lane-row form.
template <typename T, int D, bool CFL, bool NT>
__global__ void __launch_bounds__(64 * MW) ct_fluid_march_batch(const BJob* __restrict__ jobs,
                                                                const TileDesc* __restrict__ td, int njobs, int iu,
                                                                int ib)
{
    const int j = find_job(td, njobs, blockIdx.x);
    const BJob& J = jobs[j];
    const Grid g = J.g;
    const unsigned lb = blockIdx.x - td[j].first;
    ct_fluid_march_body<T, D, CFL, NT>(static_cast<const T*>(J.u[iu]), static_cast<T*>(J.u[iu ^ 1]),
                                   static_cast<const T*>(J.b[ib]), static_cast<T*>(J.b[ib ^ 1]), g, (T)J.gamma, J.ctl,
                                   -1.0, td[j].p0, lb, J.parts + lb);
}

template <typename T, bool CFL, bool NT>
__global__ void __launch_bounds__(256) ct_fluid_x_batch(const BJob* __restrict__ jobs,
                                                        const TileDesc* __restrict__ td, int njobs, int iu, int ib)
{
    const int j = find_job(td, njobs, blockIdx.x);
    const BJob& J = jobs[j];
    const Grid g = J.g;
    const unsigned lb = blockIdx.x - td[j].first;
    const T* uin = static_cast<const T*>(J.u[iu]);
    T* uout = static_cast<T*>(J.u[iu ^ 1]);
    const T* bin = static_cast<const T*>(J.b[ib]);
    T* bout = static_cast<T*>(J.b[ib ^ 1]);
    if constexpr (!kExact<T>) {
        if (td[j].p0) {
#define MHD_LROW_BFUSED(KK, WW) \
    ct_fluid_x_lrow_body<T, KK, WW, CFL, NT>(uin, uout, bin, bout, g, (T)J.gamma, J.ctl, -1.0, lb, J.parts + lb);
            MHD_BATCH_LROW_DISPATCH(td[j].p0, td[j].p1, MHD_LROW_BFUSED)
#undef MHD_LROW_BFUSED
            return;
        }
    }
    ct_fluid_x_body<T, CFL, NT>(uin, uout, bin, bout, g, (T)J.gamma, J.ctl, -1.0, lb, J.parts + lb);
}

template <typename T>
__global__ void __launch_bounds__(RB) cfl_batch(const BJob* __restrict__ jobs, const TileDesc* __restrict__ td,
                                                int njobs, int iu, int ib)
{
    const int j = find_job(td, njobs, blockIdx.x);
    const BJob& J = jobs[j];
    const Grid g = J.g;
    const unsigned lb = blockIdx.x - td[j].first;
    const unsigned nb = td[j + 1].first - td[j].first;
    cfl_body<T>(static_cast<const T*>(J.u[iu]), static_cast<const T*>(J.b[ib]), g, (T)J.gamma, lb, nb,
                J.parts + lb);
}

}  // namespace

template <typename T>
void tile_default(const Grid& g, int kind, int* p0, int* p1)
{
    *p1 = 0;
    switch (kind) {
    case KIND_CFL: *p0 = reduce_blocks(g); break;
    case KIND_FLUID_X:
    case KIND_CT_X:
    case KIND_CTFLUID_X: {   // lane-row form where it applies
        int W = 64;
        *p0 = batch_x_lrow_k<T>(g, &W);
        *p1 = *p0 ? W : 0;
        break;
    }
    case KIND_FLUID_Y: *p0 = march_chunk(g, 1, GF, kFluidMarchWaves); break;
    case KIND_FLUID_Z: *p0 = march_chunk(g, 2, GF, kFluidMarchWaves); break;
    case KIND_CT_Y: *p0 = march_chunk(g, 1, GB, kCtMarchWaves<T>); break;
    case KIND_CT_Z: *p0 = march_chunk(g, 2, GB, kCtMarchWaves<T>); break;
    case KIND_CTFLUID_Y: *p0 = march_chunk(g, 1, GCF, kFusedMarchWaves<T>); break;
    default: *p0 = march_chunk(g, 2, GCF, kFusedMarchWaves<T>); break;
    }
}

// Candidates: march chunks of the whole pencil down to an eighth of it (never
// shorter than twice the ghost depth, which would be mostly warm-up); for the
// x sweeps the wavefront and, where it applies, the lane-row form. The CFL
// pass runs only when a batch changes and keeps its default.
template <typename T>
void tile_candidates(const Grid& g, int kind, std::vector<std::pair<int, int>>& out)
{
    out.clear();
    int d0, d1;
    tile_default<T>(g, kind, &d0, &d1);
    auto add = [&](int a, int b) {
        for (auto& c : out)
            if (c.first == a && c.second == b) return;
        out.emplace_back(a, b);
    };
    add(d0, d1);
    if (kind == KIND_FLUID_X || kind == KIND_CT_X || kind == KIND_CTFLUID_X) {
        add(0, 0);
        return;
    }
    if (kind == KIND_CFL) return;
    const int axis = (kind == KIND_FLUID_Y || kind == KIND_CT_Y || kind == KIND_CTFLUID_Y) ? 1 : 2;
    const int ghost = (kind == KIND_FLUID_Y || kind == KIND_FLUID_Z) ? GF
                      : (kind == KIND_CT_Y || kind == KIND_CT_Z) ? GB : GCF;
    const int nd = g.n[axis];
    for (int div : {1, 2, 4, 8}) {
        const int c = (nd + div - 1) / div;
        if (c == nd || c >= 2 * ghost) add(c, 0);
    }
}

template <typename T>
unsigned tile_blocks(const Grid& g, int kind, int p0, int p1)
{
    switch (kind) {
    case KIND_CFL: return (unsigned)p0;
    case KIND_FLUID_X: return p0 > 0 ? x_lrow_blocks(g, p1) : x_wave_blocks(g);
    case KIND_CT_X: return p0 > 0 ? x_lrow_blocks(g, p1) : ct_x_wave_blocks(g);
    case KIND_FLUID_Y: return march_blocks(g, 1, p0, kMarchXWide<T, false>);
    case KIND_CT_Y: return march_blocks(g, 1, p0, kMarchXWide<T, true>);
    case KIND_FLUID_Z: return march_blocks(g, 2, p0, kMarchXWide<T, false>);
    case KIND_CT_Z: return march_blocks(g, 2, p0, kMarchXWide<T, true>);
    case KIND_CTFLUID_X: return p0 > 0 ? x_lrow_blocks(g, p1) : ct_fluid_x_blocks(g);
    case KIND_CTFLUID_Y: return march_blocks(g, 1, p0, kMarchXWide<T, true>);
    default: return march_blocks(g, 2, p0, kMarchXWide<T, true>);
    }
}

template <typename T, bool NT>
static hipError_t launch_batch_nt(int kind, bool cfl_parts, const BJob* jobs, const TileDesc* td, int njobs,
                                  unsigned nb, int iu, int ib, hipStream_t s)
{
    if (nb == 0 || njobs == 0) return hipSuccess;
    const dim3 mblock(64, MW);
    switch (kind) {
    case KIND_CFL: hipLaunchKernelGGL((cfl_batch<T>), dim3(nb), dim3(RB), 0, s, jobs, td, njobs, iu, ib); break;
    case KIND_FLUID_X:
        if (cfl_parts)
            hipLaunchKernelGGL((fluid_x_batch<T, true, NT>), dim3(nb), dim3(256), 0, s, jobs, td, njobs, iu, ib);
        else
            hipLaunchKernelGGL((fluid_x_batch<T, false, NT>), dim3(nb), dim3(256), 0, s, jobs, td, njobs, iu, ib);
        break;
    case KIND_FLUID_Y:
        if (cfl_parts)
            hipLaunchKernelGGL((fluid_march_batch<T, 1, true, NT>), dim3(nb), mblock, 0, s, jobs, td, njobs, iu, ib);
        else
            hipLaunchKernelGGL((fluid_march_batch<T, 1, false, NT>), dim3(nb), mblock, 0, s, jobs, td, njobs, iu, ib);
        break;
    case KIND_FLUID_Z:
        if (cfl_parts)
            hipLaunchKernelGGL((fluid_march_batch<T, 2, true, NT>), dim3(nb), mblock, 0, s, jobs, td, njobs, iu, ib);
        else
            hipLaunchKernelGGL((fluid_march_batch<T, 2, false, NT>), dim3(nb), mblock, 0, s, jobs, td, njobs, iu, ib);
        break;
    case KIND_CT_X:
        hipLaunchKernelGGL((ct_x_batch<T, NT>), dim3(nb), dim3(256), 0, s, jobs, td, njobs, iu, ib);
        break;
    case KIND_CT_Y: hipLaunchKernelGGL((ct_march_batch<T, 1, NT>), dim3(nb), mblock, 0, s, jobs, td, njobs, iu, ib); break;
    case KIND_CT_Z: hipLaunchKernelGGL((ct_march_batch<T, 2, NT>), dim3(nb), mblock, 0, s, jobs, td, njobs, iu, ib); break;
    case KIND_CTFLUID_X:
        if (cfl_parts)
            hipLaunchKernelGGL((ct_fluid_x_batch<T, true, NT>), dim3(nb), dim3(256), 0, s, jobs, td, njobs, iu, ib);
        else
            hipLaunchKernelGGL((ct_fluid_x_batch<T, false, NT>), dim3(nb), dim3(256), 0, s, jobs, td, njobs, iu, ib);
        break;
    case KIND_CTFLUID_Y:
        if (cfl_parts)
            hipLaunchKernelGGL((ct_fluid_march_batch<T, 1, true, NT>), dim3(nb), mblock, 0, s, jobs, td, njobs, iu, ib);
        else
            hipLaunchKernelGGL((ct_fluid_march_batch<T, 1, false, NT>), dim3(nb), mblock, 0, s, jobs, td, njobs, iu, ib);
        break;
    case KIND_CTFLUID_Z:
        if (cfl_parts)
            hipLaunchKernelGGL((ct_fluid_march_batch<T, 2, true, NT>), dim3(nb), mblock, 0, s, jobs, td, njobs, iu, ib);
        else
            hipLaunchKernelGGL((ct_fluid_march_batch<T, 2, false, NT>), dim3(nb), mblock, 0, s, jobs, td, njobs, iu, ib);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// A batched launch sweeps the states of all its problems: the cache policy of
// its accesses follows their total size, as for one grid of that size.
template <typename T>
hipError_t launch_batch(int kind, bool cfl_parts, const BJob* jobs, const TileDesc* td, int njobs, unsigned nb,
                        int iu, int ib, hipStream_t s, long long cells)
{
    if (8 * cells * (long long)sizeof(T) > kNtStateBytes)
        return launch_batch_nt<T, true>(kind, cfl_parts, jobs, td, njobs, nb, iu, ib, s);
    return launch_batch_nt<T, false>(kind, cfl_parts, jobs, td, njobs, nb, iu, ib, s);
}

}  // namespace mhd

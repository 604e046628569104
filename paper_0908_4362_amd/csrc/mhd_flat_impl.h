// Field sweep along an axis of one cell (d = y or z of 2D and 1D grids), in
// closed form. Kept apart from the marching kernels: it never runs on grids
// whose three axes all have more than one cell.
#pragma once
#include "mhd_kernels_impl.h"

namespace mhd {
namespace {

// Every cell of an EMF pencil along d is the same cell, so the marching
// pipeline (smoothing, first-order upwind EMF, half step, limited slope,
// second-order EMF; Sec. 3 and Alg. 2) sees a constant input and, after the
// eight cells of its latency (its 2 x 4 ghost cells cover them), holds a fixed
// point: smoothed velocity V = (v + 2v + v) / 4, first- and second-order EMFs
// Q = V B (every difference along the pencil an exact zero, so the half step
// keeps B and the limited slope is +0), and G = Q + 0 or Q - 0 by the sign of
// the edge velocity (V + V) / 2. This kernel evaluates that fixed point
// directly, one thread per cell, with the march's expressions, so for finite
// EMFs its bits are the march's (batched solves, which keep the march, are
// tested bitwise against it): the advected components keep their value
// (B - dt (G - G)) and B_d takes the constraint update from the four pencils.
template <typename T>
__device__ __forceinline__ T emf_fixed_point(T vhat, T B)
{
    const T v = T(0.25) * (vhat + T(2) * vhat + vhat);
    const T q = v * B;
    const T e = T(0.5) * (v + v);
    return e > T(0) ? q + T(0) : q - T(0);
}

template <typename T, int D>
__global__ void __launch_bounds__(256) ct_flat(const T* __restrict__ uf, const T* __restrict__ bin,
                                               T* __restrict__ bout, Grid g, const Ctl* __restrict__ ctl,
                                               double dt_arg)
{
    constexpr int E = (D + 1) % 3, F = (D + 2) % 3;
    constexpr int TA = (D == 1) ? 2 : 1;
    constexpr bool T_IS_E = (E == TA);
    const long long N = g.N;
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= N) return;
    const int nx = g.n[0], ny = g.n[1];
    const int i = (int)(c % nx);
    const long long rest = c / nx;
    const int tcv = (TA == 1) ? (int)(rest % ny) : (int)(rest / ny);   // the one of j, k that is not along d
    const int nt = g.n[TA];
    const long long st = (TA == 1) ? (long long)nx : (long long)nx * ny;
    const long long xp = wrap_idx(i + 1, nx, g.bc) - i;
    const long long xm_ = wrap_idx(i - 1, nx, g.bc) - i;
    const long long lo = (long long)(wrap_idx(tcv - 1, nt, g.bc) - tcv) * st;
    const long long hi = (long long)(wrap_idx(tcv + 1, nt, g.bc) - tcv) * st;
    const T* rho = uf;
    const T* md = uf + (1 + D) * N;
    const T* BT = bin + (T_IS_E ? E : F) * N;
    const T* BX = bin + (T_IS_E ? F : E) * N;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;

    const T r0 = rho[c], m0 = md[c];
    const T bto = BT[c], bxo = BX[c];
    const T bd = bin[D * N + c];
    const T Gt0 = emf_fixed_point(qdiv(md[c + lo] + m0, rho[c + lo] + r0), bto);
    const T Gt1 = emf_fixed_point(qdiv(m0 + md[c + hi], r0 + rho[c + hi]), BT[c + hi]);
    const T Gx0 = emf_fixed_point(qdiv(md[c + xm_] + m0, rho[c + xm_] + r0), bxo);
    const T Gx1 = emf_fixed_point(qdiv(m0 + md[c + xp], r0 + rho[c + xp]), BX[c + xp]);
    const T Ge0 = T_IS_E ? Gt0 : Gx0, Ge1 = T_IS_E ? Gt1 : Gx1;
    const T Gf0 = T_IS_E ? Gx0 : Gt0, Gf1 = T_IS_E ? Gx1 : Gt1;
    const T be = T_IS_E ? bto : bxo, bfv = T_IS_E ? bxo : bto;
    if (frozen) {
        bout[E * N + c] = be;
        bout[F * N + c] = bfv;
        bout[D * N + c] = bd;
    } else {
        bout[E * N + c] = be - dt * (Ge0 - Ge0);
        bout[F * N + c] = bfv - dt * (Gf0 - Gf0);
        bout[D * N + c] = (bd + dt * (Ge1 - Ge0)) + dt * (Gf1 - Gf0);
    }
}

}  // namespace

template <typename T>
hipError_t launch_ct_flat(int axis, const T* u, const T* b_in, T* b_out, Grid g, const Ctl* ctl, double dt,
                          hipStream_t s)
{
    if (axis < 1 || axis > 2 || g.n[axis] != 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((g.N + 255) / 256)), block(256);
    if (axis == 1)
        hipLaunchKernelGGL((ct_flat<T, 1>), grid, block, 0, s, u, b_in, b_out, g, ctl, dt);
    else
        hipLaunchKernelGGL((ct_flat<T, 2>), grid, block, 0, s, u, b_in, b_out, g, ctl, dt);
    return hipGetLastError();
}
}  // namespace mhd

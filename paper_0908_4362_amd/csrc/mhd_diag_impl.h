// Derived fields of a state for headless diagnostics, in place of the paper's
// on-screen rendering of the density, pressure and field (Sec. 8): gas
// pressure, magnetic pressure, speed, CFL speed and the cell divergence of B,
// for the whole grid or for one plane of it; and the check of an input state
// (every value finite, density positive).
#pragma once
#include "mhd_kernels_impl.h"

namespace mhd {
namespace {

template <typename T>
__global__ void __launch_bounds__(256) diag_kernel(const T* __restrict__ u, const T* __restrict__ b, Grid g,
                                                   T gamma, int kind, int axis, int index, T* __restrict__ out,
                                                   long long nout)
{
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const long long N = g.N;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nout;
         q += (long long)gridDim.x * blockDim.x) {
        int i, j, k;
        if (axis == 0) {
            i = index;
            j = (int)(q % ny);
            k = (int)(q / ny);
        } else if (axis == 1) {
            i = (int)(q % nx);
            j = index;
            k = (int)(q / nx);
        } else if (axis == 2) {
            i = (int)(q % nx);
            j = (int)(q / nx);
            k = index;
        } else {
            i = (int)(q % nx);
            j = (int)((q / nx) % ny);
            k = (int)(q / ((long long)nx * ny));
        }
        const long long c = i + (long long)nx * (j + (long long)ny * k);
        const long long cx = wrap_idx(i + 1, nx, g.bc) + (long long)nx * (j + (long long)ny * k);
        const long long cy = i + (long long)nx * (wrap_idx(j + 1, ny, g.bc) + (long long)ny * k);
        const long long cz = i + (long long)nx * (j + (long long)ny * wrap_idx(k + 1, nz, g.bc));
        T v;
        if (kind == 3) {   // cell divergence of the face field (upper minus lower faces)
            v = ((b[cx] - b[c]) + (b[N + cy] - b[N + c])) + (b[2 * N + cz] - b[2 * N + c]);
        } else {
            const T bx = T(0.5) * (b[c] + b[cx]);
            const T by = T(0.5) * (b[N + c] + b[N + cy]);
            const T bz = T(0.5) * (b[2 * N + c] + b[2 * N + cz]);
            const T bb = bx * bx + by * by + bz * bz;
            const T rho = u[c];
            const T vx = u[N + c] / rho, vy = u[2 * N + c] / rho, vz = u[3 * N + c] / rho;
            const T vv = vx * vx + vy * vy + vz * vz;
            if (kind == 0)
                v = (gamma - T(1)) * (u[4 * N + c] - T(0.5) * rho * vv - T(0.5) * bb);
            else if (kind == 1)
                v = T(0.5) * bb;
            else if (kind == 2)
                v = sqrt(vv);
            else
                v = cfl_speed<T>(rho, u[N + c], u[2 * N + c], u[3 * N + c], u[4 * N + c], bx, by, bz, gamma);
        }
        out[q] = v;
    }
}

// Input check: a non-finite value in any field or a non-positive density
// latches status -1 in the control block (every offending thread stores the
// same value; the status was cleared before the launch).
template <typename T>
__global__ void __launch_bounds__(256) validate_kernel(const T* __restrict__ u, const T* __restrict__ b, long long N,
                                                       Ctl* __restrict__ ctl)
{
    bool bad = false;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < N; c += (long long)gridDim.x * blockDim.x) {
        const T rho = u[c];
        bad |= !(rho > T(0)) || !isfinite(rho);
        for (int q = 1; q < 5; q++) bad |= !isfinite(u[q * N + c]);
        for (int q = 0; q < 3; q++) bad |= !isfinite(b[q * N + c]);
    }
    if (bad) ctl->status = -1;
}

}  // namespace

template <typename T>
hipError_t launch_validate(const T* u, const T* b, long long N, Ctl* ctl, hipStream_t s)
{
    long long nb = (N + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL((validate_kernel<T>), dim3((unsigned)nb), dim3(256), 0, s, u, b, N, ctl);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diag(const T* u, const T* b, Grid g, double gamma, int kind, int axis, int index, T* out,
                       hipStream_t s)
{
    long long nout = g.N;
    if (axis == 0) nout = (long long)g.n[1] * g.n[2];
    if (axis == 1) nout = (long long)g.n[0] * g.n[2];
    if (axis == 2) nout = (long long)g.n[0] * g.n[1];
    long long nb = (nout + 255) / 256;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL((diag_kernel<T>), dim3((unsigned)nb), dim3(256), 0, s, u, b, g, (T)gamma, kind, axis, index,
                       out, nout);
    return hipGetLastError();
}

}  // namespace mhd

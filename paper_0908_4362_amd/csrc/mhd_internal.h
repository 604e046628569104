// Internal declarations shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mhd {

// Grid description passed by value to every kernel.
struct Grid {
    int n[3];       // cells along x, y, z
    int bc;         // 0 periodic, 1 outflow
    long long N;    // cells per field
};

// Device-resident control block: time-step state of one solver.
struct Ctl {
    double dt;                      // step in use by the sweeps
    double t;                       // simulation time (advanced by the CFL kernel)
    double t_stop;                  // < 0: none
    double cmax;                    // last c_max
    unsigned long long max_bits;    // running max of non-negative values (ordered bit pattern)
    unsigned int blocks_done;       // arrival counter of the reduction
    int status;                     // 0 ok, -4 non-finite c_max (latched)
    unsigned long long div_bits;    // running max for the div B reduction
    unsigned int div_blocks_done;
    int pad;
};

// Launchers (return hipSuccess or the launch error).
template <typename T>
hipError_t launch_cfl(const T* u, const T* b, Grid g, double gamma, double cfl, Ctl* ctl, hipStream_t s);
template <typename T>
hipError_t launch_cmax_only(const T* u, const T* b, Grid g, double gamma, Ctl* ctl, hipStream_t s);
// Conserved fields u = (rho, m_x, m_y, m_z, E) and face fields b = (B_x, B_y, B_z)
// are each stored field-major with N cells per field. Sweeps read dt and the
// status word from the control block; a non-negative dt argument replaces the
// control block's dt (sub-operation calls).
template <typename T>
hipError_t launch_fluid(int axis, const T* u_in, T* u_out, const T* b, Grid g, double gamma, const Ctl* ctl,
                        double dt, hipStream_t s);
template <typename T>
hipError_t launch_ct(int axis, const T* u, const T* b_in, T* b_out, Grid g, const Ctl* ctl, double dt,
                     hipStream_t s);
template <typename T>
hipError_t launch_divb(const T* b, Grid g, Ctl* ctl, hipStream_t s);

}  // namespace mhd

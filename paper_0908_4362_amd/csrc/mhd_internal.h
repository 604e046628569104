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
    double dt;      // step in use by the sweeps
    double t;       // simulation time (advanced when dt is set)
    double t_stop;  // < 0: none
    double cmax;    // c_max of the current state (from the last reduction)
    double divb;    // result of the last div B reduction
    int status;     // 0 ok, -4 non-finite c_max (latched)
    int pad;
};

// Grid-wide maxima are reduced in two levels: a producing kernel stores one
// maximum per workgroup (ordered bit patterns of non-negative doubles) in a
// parts array, then launch_finish reduces them with one workgroup.
size_t reduce_capacity(const Grid& g);   // largest number of parts any launch writes
hipError_t launch_finish(const unsigned long long* parts, int nparts, int what, double cfl, Ctl* ctl,
                         hipStream_t s);  // what 0: c_max (and the dt rule if cfl > 0); 1: div B

// Producers (return hipSuccess or the launch error; *nparts = parts written).
template <typename T>
hipError_t launch_cfl(const T* u, const T* b, Grid g, double gamma, unsigned long long* parts, int* nparts,
                      hipStream_t s);
template <typename T>
hipError_t launch_divb(const T* b, Grid g, unsigned long long* parts, int* nparts, hipStream_t s);

// Sweeps: conserved fields u = (rho, m_x, m_y, m_z, E) and face fields
// b = (B_x, B_y, B_z), each field-major with N cells per field. A sweep reads
// the status word and, unless dt >= 0 is given, dt from the control block.
// With parts non-null the fluid sweep also stores per-workgroup maxima of the
// CFL speed of the state it writes.
template <typename T>
hipError_t launch_fluid(int axis, const T* u_in, T* u_out, const T* b, Grid g, double gamma, const Ctl* ctl,
                        double dt, unsigned long long* parts, int* nparts, hipStream_t s);
template <typename T>
hipError_t launch_ct(int axis, const T* u, const T* b_in, T* b_out, Grid g, const Ctl* ctl, double dt,
                     hipStream_t s);

}  // namespace mhd

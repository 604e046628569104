// Internal declarations shared by the HIP kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>
#include <vector>

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
    int status;     // 0 ok, -4 non-finite c_max, -1 invalid input state (latched)
    int nparts;     // per-workgroup c_max slots the last producing launch wrote
};

// Error reporting of the C ABI: record a message for mhd_last_error() and
// return code (report_hip: MHD_ERR_DEVICE with the HIP error text).
int report(int code, const char* msg);
int report_hip(hipError_t e, const char* where);

// Grid-wide maxima are reduced in two levels: a producing kernel stores one
// maximum per workgroup (ordered bit patterns of non-negative doubles) in a
// parts array, then launch_finish reduces them with one workgroup. A c_max
// producer of the plain solver also stores its slot count in ctl->nparts, and
// the finisher of c_max reads the count from there, so a step replayed from a
// graph reduces exactly the slots the previous producer wrote, whichever
// launch that was (a fluid sweep of any axis, or the standalone pass).
size_t reduce_capacity(const Grid& g);   // largest number of parts any launch writes
int reduce_slots(const Grid& g);         // parts launch_cfl and launch_divb write (at most 8192)
// what 0: c_max over ctl->nparts slots (and the dt rule if cfl > 0);
// what 1: max |div B| over nparts slots into ctl->divb
hipError_t launch_finish(const unsigned long long* parts, int nparts, int what, double cfl, Ctl* ctl,
                         hipStream_t s);

// Producers (return hipSuccess or the launch error). launch_cfl stores its
// slot count in ctl->nparts on the device; launch_divb returns it in *nparts.
template <typename T>
hipError_t launch_cfl(const T* u, const T* b, Grid g, double gamma, unsigned long long* parts, Ctl* ctl,
                      hipStream_t s);
template <typename T>
hipError_t launch_divb(const T* b, Grid g, unsigned long long* parts, int* nparts, hipStream_t s);

// Sweeps: conserved fields u = (rho, m_x, m_y, m_z, E) and face fields
// b = (B_x, B_y, B_z), each field-major with N cells per field. A sweep reads
// the status word and, unless dt >= 0 is given, dt from the control block.
// With parts non-null the fluid sweep also stores per-workgroup maxima of the
// CFL speed of the state it writes, and its slot count in ctl->nparts.
template <typename T>
hipError_t launch_fluid(int axis, const T* u_in, T* u_out, const T* b, Grid g, double gamma, Ctl* ctl,
                        double dt, unsigned long long* parts, hipStream_t s);
template <typename T>
hipError_t launch_ct(int axis, const T* u, const T* b_in, T* b_out, Grid g, const Ctl* ctl, double dt,
                     hipStream_t s);
// Reverse L_d along any axis of a periodic grid in one launch: the field
// update (reads u, b_in; writes b_out) then the fluid update on the new field
// (reads u_in; writes u_out), the same results as launch_ct then
// launch_fluid. With parts non-null the fluid part stores the c_max slots.
template <typename T>
hipError_t launch_ct_fluid(int axis, const T* u_in, T* u_out, const T* b_in, T* b_out, Grid g, double gamma,
                           Ctl* ctl, double dt, unsigned long long* parts, hipStream_t s);
// Whether the fused launch is faster than the two launches for this axis.
template <typename T>
bool fused_reverse_pays(const Grid& g, int axis);
// The field sweep along axis 1 or 2 when that axis has one cell: the fixed
// point of the marching pipeline, evaluated per cell (same results bit for
// bit, one pass over the fields instead of a warm-up per chunk).
template <typename T>
hipError_t launch_ct_flat(int axis, const T* u, const T* b_in, T* b_out, Grid g, const Ctl* ctl, double dt,
                          hipStream_t s);

// ---------------------------------------------------------------------------
// Batched launches: one launch runs one sub-operation for many independent
// problems; workgroup w of the launch belongs to the problem whose range
// [first, next first) holds w.

// Launch kinds (numbered as the MHD_K_* timing kinds of the C ABI).
enum {
    KIND_CFL = 0,
    KIND_FLUID_X,
    KIND_FLUID_Y,
    KIND_FLUID_Z,
    KIND_CT_X,
    KIND_CT_Y,
    KIND_CT_Z,
    KIND_CTFLUID_X,   // reverse L_d fused (field update, then fluid update), periodic grids
    KIND_CTFLUID_Y,
    KIND_CTFLUID_Z,
    KIND_COUNT
};

// One problem of a batch as the batched kernels see it.
struct BJob {
    void* u[2];                  // conserved fields, ping-pong copies (5 N elements each)
    void* b[2];                  // face fields, ping-pong copies (3 N elements each)
    Ctl* ctl;                    // the problem's control block (dt, t, stop time, status)
    unsigned long long* parts;   // per-workgroup maxima of this problem
    Grid g;
    double gamma;
};

// Workgroups and tile parameters of one problem in one batched launch:
// p0 = chunk length (y/z sweeps), cells per lane of the lane-row form or 0
// for the wavefront form (x sweeps), or workgroup count (CFL); p1 = 0.
struct TileDesc {
    unsigned first;
    int p0, p1;
    int pad;
};

// Tiles of one kind for a problem: the plain solver's choice, the
// candidates the autotuner may time, and the workgroup count.
template <typename T>
void tile_default(const Grid& g, int kind, int* p0, int* p1);
template <typename T>
void tile_candidates(const Grid& g, int kind, std::vector<std::pair<int, int>>& out);
template <typename T>
unsigned tile_blocks(const Grid& g, int kind, int p0, int p1);

// One batched sub-operation over njobs problems (tables in device memory,
// nblocks = last first + last count). iu / ib select the ping-pong copies
// read (the other copy is written). With cfl_parts a fluid sweep also stores
// per-workgroup CFL maxima into each problem's parts. cells: the problems'
// total cell count, which picks the cache policy of the launch's accesses.
template <typename T>
hipError_t launch_batch(int kind, bool cfl_parts, const BJob* jobs, const TileDesc* td, int njobs, unsigned nblocks,
                        int iu, int ib, hipStream_t s, long long cells);
// Per-problem second level of the c_max reduction (td: the producing launch's
// table) and the dt rule of each problem.
hipError_t launch_finish_batch(const BJob* jobs, const TileDesc* td, int njobs, double cfl, hipStream_t s);

// Derived field `kind` (0 gas pressure, 1 magnetic pressure, 2 speed, 3 cell
// divergence of B, 4 CFL speed) for the whole grid (axis < 0, N values) or
// for the plane axis = index (values in the order of the two other axes, the
// lower one fastest), into out.
template <typename T>
hipError_t launch_diag(const T* u, const T* b, Grid g, double gamma, int kind, int axis, int index, T* out,
                       hipStream_t s);

// Input check of a state (u: 5 N, b: 3 N elements): sets ctl->status = -1 if
// any value is not finite or some density is not positive.
template <typename T>
hipError_t launch_validate(const T* u, const T* b, long long N, Ctl* ctl, hipStream_t s);

}  // namespace mhd

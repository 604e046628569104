/*
 * mhd.h - C ABI of the MI355X (gfx950) ideal-MHD time-step library.
 *
 * The library advances the ideal-MHD equations (Wong et al., Sec. 3: the
 * conservation laws for rho, rho v, B, E with mu = 1, P* = p + B^2/2 and
 * p = (gamma - 1)(E - rho v^2/2 - B^2/2)) on a 3D Cartesian grid of unit cells
 * with Pen et al.'s relaxing-TVD scheme in dimensionally split sweeps and a
 * constrained-transport update of the face-centred field that keeps div B at
 * round-off. The problem statement follows the paper's program flow (Sec. 4.2):
 * build an initial state on the host, copy it in, advance with a Courant
 * number, read it back.
 *
 * State layout (every state buffer passed across this ABI):
 *   one contiguous array of 8 * nx * ny * nz elements of the handle's dtype
 *   (float for MHD_F32, double for MHD_F64), field-major in the order
 *   rho, m_x, m_y, m_z, E, B_x, B_y, B_z (m = rho v, E total energy density);
 *   within a field x is fastest: element (i, j, k) is at i + nx * (j + ny * k).
 *   B_d(i, j, k) is the field on the lower d-face of cell (i, j, k)
 *   (eq. equat_b). Cells have unit width, so times are in cell-crossing units:
 *   a physical time t on a box of n cells per unit length is t * n.
 *
 * Arithmetic: MHD_F64 evaluates every expression of the scheme in IEEE double
 * precision in a fixed order, without fused multiply-adds, with correctly
 * rounded quotients (for operands in the normal range) and square roots, so
 * it equals a plain serial evaluation bit for bit. MHD_F32 fuses a multiply and
 * an add within one expression and uses the hardware reciprocal and square root
 * (1 ulp). In both, a step is deterministic and its result does not depend on
 * how the work is laid out on the device (grid shape of the launches, march
 * chunks, batch tiles): a batched or served problem gets the same bits as a
 * plain handle.
 *
 * Return codes: MHD_OK (0) or a negative MHD_ERR_* value; after an error,
 * mhd_last_error() returns a message (thread-local). No exception crosses the
 * ABI. A handle is not thread-safe; distinct handles are independent. All
 * device work of a handle runs on its stream (the null stream by default).
 * Device pointers are HIP device addresses on the current device.
 */
#ifndef MHD_H
#define MHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mhd_solver mhd_t;

enum {
    MHD_OK = 0,
    MHD_ERR_ARG = -1,       /* invalid argument (null pointer, size, value)     */
    MHD_ERR_OOM = -2,       /* device allocation failed                         */
    MHD_ERR_DEVICE = -3,    /* a HIP runtime call failed                        */
    MHD_ERR_NONFINITE = -4  /* c_max was NaN, infinite or not positive          */
};

enum { MHD_BC_PERIODIC = 0, MHD_BC_OUTFLOW = 1 };
enum { MHD_F32 = 0, MHD_F64 = 1 };

/* Create a solver for an nx x ny x nz grid (each >= 1, at most 2^36 cells in
 * all; sizes need not be powers of two), adiabatic index gamma > 1, boundary
 * condition bc applied on
 * every axis (periodic wrap, or outflow = zero-gradient copy of cell and face
 * values beyond the edge) and arithmetic type dtype. The paper's program
 * works on a regular Cartesian grid in single or double precision and keeps
 * the eight components in eight arrays in device memory (Sec. 4, its opening
 * and Sec. 4.1); this call is the set-up of steps 1-2 of its program flow
 * (Sec. 4.2). The handle owns its device memory: two ping-pong copies of the
 * state plus a few scalars. The state starts undefined; call mhd_set_state
 * before stepping. */
int mhd_create(int nx, int ny, int nz, double gamma, int bc, int dtype, mhd_t** out);

/* Release the handle and its device memory (null is accepted). */
int mhd_destroy(mhd_t* h);

/* Use a caller-owned HIP stream (hipStream_t passed as void*; null = the
 * null stream) for all later work of this handle. Waits for the work already
 * issued on the previous stream, so the handle's operations stay ordered. */
int mhd_set_stream(mhd_t* h, void* stream);

/* Replay full steps from HIP graphs (enable = 1, the default) or issue every
 * launch directly (0). Replay applies on a stream other than the null
 * stream, with per-kernel timing off: each sweep order's step (dt rule and
 * 12 sweeps) is captured once and relaunched, which removes the per-launch
 * host cost that dominates small grids. Results are identical either way. */
int mhd_set_graphs(mhd_t* h, int enable);

/* Run each reverse L_d of a periodic grid (field update, then fluid update,
 * Sec. 4.3) as one launch that keeps the new field on the chip: mode 1 (the
 * default) where that is the faster form for the grid (always along x; along
 * y and z where the grid is large enough for long marching chunks), 2 on every
 * axis, 0 never (two launches). Results are identical in every mode; grids
 * with outflow boundaries always take two launches. */
int mhd_set_fusion(mhd_t* h, int mode);

/* Copy a state in (layout above) from host memory or from device memory
 * (step 3 of the program flow of Sec. 4.2: the initial u and face B to
 * device memory; with t set to 0 as in step 2);
 * resets t = 0 and the step counter s = 0, then checks it on the device and
 * returns MHD_ERR_ARG if a value is not finite or a density is not positive
 * (the handle then refuses to step, with MHD_ERR_ARG, until a valid state is
 * set). Both variants return when the copy and the check are done. The
 * caller keeps ownership of the buffer. */
int mhd_set_state(mhd_t* h, const void* host_state);
int mhd_set_state_device(mhd_t* h, const void* dev_state);

/* Copy the current state out (layout above) to host memory (synchronises the
 * stream) or to device memory (asynchronous on the handle's stream): step 10
 * of the program flow of Sec. 4.2 (read u and B back). */
int mhd_get_state(mhd_t* h, void* host_state);
int mhd_get_state_device(mhd_t* h, void* dev_state);

/* Advance n >= 0 full steps with Courant number 0 < cfl <= 1 (Sec. 3,
 * eq. equat_CFL; Sec. 4.2). One full step computes c_max and
 * dt = cfl / c_max, then applies the forward sweep L_z L_y L_x and the
 * reverse sweep L_x L_y L_z (each L_d = fluid_d, B_{e->d}, B_{f->d}; reversed
 * inside the reverse sweep), rotating the axis order with the step counter
 * s (eq. L_sequence); t advances by 2 dt. dt, t and s stay on the device; the
 * call reads one status word back at its end. With a stop time set, the last
 * dt is clipped so that t lands on it, and later steps do nothing.
 * Returns MHD_ERR_NONFINITE if some step met a NaN/inf/non-positive c_max;
 * the state is then the one that step started from, and stays frozen until
 * mhd_set_state. Returns MHD_ERR_ARG (nothing advances) while the state set
 * last is one mhd_set_state rejected. */
int mhd_step(mhd_t* h, int n, double cfl);

/* max over cells of |sum_d (B_d(c + e_d) - B_d(c))| in unit cells: the
 * discrete div B of the face field of eq. equat_b, which the constrained
 * transport of Sec. 3 keeps at machine precision (the constraint div B = 0
 * stated with the MHD equations, Sec. 3). With outflow boundaries only cells
 * whose upper faces are stored are counted (axes of size 1 contribute
 * nothing). Synchronises the stream. */
int mhd_divb_max(mhd_t* h, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * quantity of mhd_divb_max for a state in the caller's device memory, with no
 * handle. dev_state: 8 * nx * ny * nz elements of dtype in the state layout
 * above (only the face fields are read); bc, dtype and the sizes as in
 * mhd_create. The maximum is written, as a double, to the caller's device
 * pointer dev_out, asynchronously on stream (hipStream_t as void*, null = the
 * null stream); nothing is allocated and nothing synchronises. The reduction
 * uses a fixed device array of the library (8192 slots and a control block,
 * about 64 KiB, one copy per device, held until the process ends); every
 * grid that mhd_create accepts fits it. All calls on one device share that
 * array, so calls whose work overlaps on a device (other streams, other host
 * threads) race: order them. Errors: MHD_ERR_ARG for null pointers, sizes,
 * bc or dtype out of range; MHD_ERR_DEVICE if a launch fails. */
int mhd_divb_max_noalloc(const void* dev_state, int nx, int ny, int nz, int bc, int dtype, double* dev_out,
                         void* stream);

/* Simulation time and step counter (s mod 3 selects the sweep order). */
int mhd_get_time(mhd_t* h, double* t, int64_t* s);
int mhd_set_time(mhd_t* h, double t, int64_t s);

/* Stop time in the same units as t; a negative value clears it. */
int mhd_set_stop_time(mhd_t* h, double t_stop);

/* Message describing the last error of this thread ("" if none). */
const char* mhd_last_error(void);

/* ---- sub-operations of the step (the paper's named operations), for
 * checking and profiling them one at a time. Each runs asynchronously on the
 * handle's stream and leaves t and s unchanged. ---- */

/* fluid_d (Alg. 1): relaxing-TVD update of rho, m, E along axis d (0, 1, 2)
 * with the field frozen, time step dt >= 0. */
int mhd_fluid_sweep(mhd_t* h, int axis, double dt);

/* B_{e->d} then B_{f->d} (Alg. 2): advection of the two transverse face
 * components along axis d and constraint update of B_d with the same EMFs,
 * fluid frozen, time step dt >= 0. */
int mhd_ct_sweep(mhd_t* h, int axis, double dt);

/* Global maximum of the CFL speed of eq. equat_CFL over all cells
 * (synchronises; NaN if some cell is not finite). */
int mhd_cmax(mhd_t* h, double* out);

/* One full step with a caller-given dt and the sweep order of step index
 * s_order (eq. L_sequence); t and s are not changed. */
int mhd_step_dt(mhd_t* h, double dt, int64_t s_order);

/* ---- per-kernel timing: HIP events recorded on the handle's stream around
 * every kernel launch, grouped by kind. ---- */
enum {
    MHD_K_CFL = 0,       /* max-speed reduction passes and dt rule           */
    MHD_K_FLUID_X = 1,   /* fluid_d, d = x, y, z: MHD_K_FLUID_X + d          */
    MHD_K_FLUID_Y = 2,
    MHD_K_FLUID_Z = 3,
    MHD_K_CT_X = 4,      /* field update along d: MHD_K_CT_X + d             */
    MHD_K_CT_Y = 5,
    MHD_K_CT_Z = 6,
    MHD_K_CTFLUID_X = 7, /* reverse L_d fused into one launch (field update  */
    MHD_K_CTFLUID_Y = 8, /* then fluid update): MHD_K_CTFLUID_X + d           */
    MHD_K_CTFLUID_Z = 9,
    MHD_K_COUNT = 10
};

/* Start (enable = 1, clears the totals) or stop (0) recording. */
int mhd_timing(mhd_t* h, int enable);

/* Total milliseconds and number of launches recorded for one kernel kind
 * (synchronises the stream). */
int mhd_timing_read(mhd_t* h, int kind, double* total_ms, int64_t* launches);

/* Number of device bytes a handle of this size holds. */
size_t mhd_state_bytes(int nx, int ny, int nz, int dtype);

/* Size of a caller-owned workspace that can hold all of a handle's device
 * memory (two state copies, control block, reduction slots); 0 for invalid
 * arguments. */
size_t mhd_workspace_bytes(int nx, int ny, int nz, int dtype);

/* Move the handle into a caller-owned device buffer (e.g. memory a PyTorch
 * allocator owns) of at least mhd_workspace_bytes bytes, 256-byte aligned:
 * the handle releases its own allocations and never frees the workspace,
 * which must outlive the handle. The state is then undefined, t = 0 and
 * s = 0 (call mhd_set_state); MHD_ERR_ARG for a null, misaligned or too
 * small buffer (the handle is then unchanged). Synchronises the stream. */
int mhd_bind_workspace(mhd_t* h, void* dev, size_t bytes);

/* Headless diagnostics: the derived fields one would render (the paper shows
 * density, gas pressure and field images, Sec. 5 and Sec. 8), computed on
 * the device from the current state with the centred field of eq. equat_b
 * averaged from the two faces of each cell:
 *   MHD_D_PRESSURE           p = (gamma - 1)(E - rho v^2 / 2 - b^2 / 2)
 *   MHD_D_MAGNETIC_PRESSURE  b^2 / 2
 *   MHD_D_SPEED              |v|
 *   MHD_D_DIVB               sum over d of B_d(upper face) - B_d(lower face)
 *                            (faces beyond the edge through the boundary map)
 *   MHD_D_CFL_SPEED          max_d |v_d| + sqrt(|gamma p + b^2| / rho)
 * axis < 0: the whole grid, nx*ny*nz values in the state's cell order;
 * axis = 0, 1 or 2: the plane x, y or z = index (0 <= index < n_axis), in the
 * cell order of the two remaining axes (the lower-numbered one fastest).
 * dev_out: device buffer of the handle's dtype, written asynchronously on the
 * handle's stream. */
enum {
    MHD_D_PRESSURE = 0,
    MHD_D_MAGNETIC_PRESSURE = 1,
    MHD_D_SPEED = 2,
    MHD_D_DIVB = 3,
    MHD_D_CFL_SPEED = 4,
    MHD_D_COUNT = 5
};
int mhd_diagnostic(mhd_t* h, int kind, int axis, int index, void* dev_out);

#ifdef __cplusplus
}
#endif

#endif /* MHD_H */

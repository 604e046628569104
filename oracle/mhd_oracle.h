/*
 * CPU oracle for one full time step of the relaxing-TVD + constrained-transport
 * ideal-MHD scheme (Wong et al., "Efficient magnetohydrodynamic simulations on
 * graphics processing units with CUDA", Sec. 3).
 *
 * TEST INFRASTRUCTURE ONLY. This code is the slow, serial, FP64 reference that
 * the GPU path is checked against (a build with -fopenmp shares the pencils
 * of each sweep among threads and gives the same bits). Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code, header,
 * table or helper with the GPU library.
 *
 * State layout (shared convention with the public API, re-declared here):
 * one contiguous array of 8 * nx * ny * nz doubles, field-major in the order
 * rho, m_x, m_y, m_z, E, B_x, B_y, B_z; within a field x is fastest:
 * index = i + nx * (j + ny * k). B_d(i,j,k) is the face value at the
 * lower d-face of cell (i,j,k) (Sec. 3, eq. equat_b). Cells have unit width.
 */
#ifndef MHD_ORACLE_H
#define MHD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Boundary condition applied on every axis: 0 = periodic wrap,
 * 1 = outflow (zero-gradient clamp of cell and face arrays). */
typedef struct {
    int n[3];
    double gamma;
    int bc;
} orc_grid;

/* van Leer limiter, eq. limiter; zero unless a*b > 0. */
double orc_vanleer(double a, double b);

/* Flux of eq. flux rotated to the sweep axis, and the per-cell freezing speed.
 * u = (rho, m_normal, m_t1, m_t2, E), b = (b_normal, b_t1, b_t2) centred. */
void orc_flux_speed(const double* u, const double* b, double gamma, double* F, double* c);

/* fluid_d (Alg. 1): out = state after the fluid update along axis d with B frozen. */
void orc_fluid_sweep(const orc_grid* g, const double* in, double* out, int d, double dt);

/* B_{e->d} then B_{f->d} (Alg. 2): advection of both transverse face components
 * along d and the constraint update of B_d, fluid frozen. */
void orc_ct_sweep(const orc_grid* g, const double* in, double* out, int d, double dt);

/* Global maximum of the CFL speed of eq. equat_CFL (NaN if any cell is NaN). */
double orc_cmax(const orc_grid* g, const double* s);

/* Time-step rule. t_stop < 0 means "no stop time". Returns 0 on success,
 * -4 if c_max is not a positive finite number. */
int orc_dt(double cmax, double cfl, double t, double t_stop, double* dt, double* t_new);

/* One full step with a given dt and sweep-order index s (eq. L_sequence). */
void orc_step_dt(const orc_grid* g, double* s, double dt, long long step);

/* One full step: CFL, forward and reverse sweeps, t += 2 dt, step += 1.
 * Returns 0 or -4 (non-finite c_max; state untouched). */
int orc_step(const orc_grid* g, double* s, double cfl, double t_stop, double* t, long long* step);

/* max |div B| over cells whose faces are all stored (all cells if periodic). */
double orc_divb_max(const orc_grid* g, const double* s);

/* Threads of the OpenMP build (n > 0 sets them); returns the count in use,
 * 1 for the serial build. Results do not depend on it. */
int orc_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif

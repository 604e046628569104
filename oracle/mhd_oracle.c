/*
 * CPU oracle: plain serial FP64 implementation of one full step of the
 * relaxing-TVD fluid update plus constrained-transport field update of
 * Wong et al. (Sec. 3 and Sec. 4.3, Alg. 1 and Alg. 2).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the GPU library. Build with
 * -ffp-contract=off and without fast-math.
 *
 * Built with -fopenmp, the independent pencils of a sweep (and the cells of
 * the two maxima) are shared among threads; each pencil's arithmetic is the
 * same code in the same order, and maxima are exact, so the threaded build
 * gives the serial build's bits. Without -fopenmp the pragmas are ignored.
 *
 * Every derived quantity (centred field, face velocity, flux, mover, limiter
 * slope, EMF) at any index, inside the grid or beyond its edge, is computed
 * from the boundary-mapped primary state (rho, m, E, face B); a derived
 * quantity is never itself wrapped or clamped. The stage-1 (half step) values
 * beyond the edge are computed the same way and are not re-bounded.
 */
#include "mhd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { RHO = 0, MX = 1, EN = 4, BX = 5 };
#define NF 8
#define GF 3 /* ghost depth of the fluid sweep (stencil of stages 1 + 2) */
#define GB 4 /* ghost depth of the field sweep (adds the 1-2-1 smoothing) */

static long ncell(const orc_grid* g) { return (long)g->n[0] * g->n[1] * g->n[2]; }

/* Boundary index map along one axis. */
static int bmap(const orc_grid* g, int axis, int i)
{
    int n = g->n[axis];
    if (g->bc == 0) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* Linear index of the (boundary-mapped) cell c. */
static long lin(const orc_grid* g, const int c[3])
{
    int i = bmap(g, 0, c[0]), j = bmap(g, 1, c[1]), k = bmap(g, 2, c[2]);
    return (long)i + (long)g->n[0] * ((long)j + (long)g->n[1] * k);
}

static const double* fld(const orc_grid* g, const double* s, int f) { return s + (long)f * ncell(g); }

double orc_vanleer(double a, double b)
{
    /* eq. limiter: 2ab/(a+b); no correction when the two half-differences of
     * eq. Delta_F have opposite signs (or one is zero). */
    double ab = a * b;
    if (ab > 0.0) return 2.0 * ab / (a + b);
    return 0.0;
}

void orc_flux_speed(const double* u, const double* b, double gamma, double* F, double* c)
{
    /* Sec. 3: P* = p + B^2/2, p = (gamma-1)(E - rho v^2/2 - B^2/2);
     * eq. flux written for the sweep axis (normal components first). */
    double rho = u[0];
    double vn = u[1] / rho, v1 = u[2] / rho, v2 = u[3] / rho;
    double bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double vv = vn * vn + v1 * v1 + v2 * v2;
    double p = (gamma - 1.0) * (u[4] - 0.5 * rho * vv - 0.5 * bb);
    double ps = p + 0.5 * bb;
    double bv = b[0] * vn + b[1] * v1 + b[2] * v2;
    F[0] = u[1];
    F[1] = u[1] * vn + ps - b[0] * b[0];
    F[2] = u[2] * vn - b[0] * b[1];
    F[3] = u[3] * vn - b[0] * b[2];
    F[4] = (u[4] + ps) * vn - b[0] * bv;
    /* freezing speed: |v_n| + sqrt(gamma p / rho + B^2 / rho), taken per cell
     * (c_n^t); the absolute value keeps it defined if the pressure goes
     * negative. */
    *c = fabs(vn) + sqrt(fabs(gamma * p + bb) / rho);
}

/* Right/left movers of eq. lr multiplied by c: r = c u^R = (c u + F)/2,
 * l = c u^L = (c u - F)/2. */
static void movers(const double* u, const double* b, double gamma, double* r, double* l)
{
    double F[5], c;
    orc_flux_speed(u, b, gamma, F, &c);
    for (int q = 0; q < 5; q++) {
        r[q] = 0.5 * (c * u[q] + F[q]);
        l[q] = 0.5 * (c * u[q] - F[q]);
    }
}

/* Limited slope of a cell-centred quantity from its two half-differences
 * (eq. Delta_F, eq. Delta_F_n). */
static double slope(double qm, double q0, double qp)
{
    return orc_vanleer((q0 - qm) / 2.0, (qp - q0) / 2.0);
}

/* out = in for a whole state (the OpenMP build copies in parallel chunks). */
static void copy_state(const orc_grid* g, const double* in, double* out)
{
    const long total = NF * ncell(g);
    const long chunk = 1L << 16;
    const long nchunks = (total + chunk - 1) / chunk;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < nchunks; c++) {
        const long lo = c * chunk, hi = lo + chunk < total ? lo + chunk : total;
        memcpy(out + lo, in + lo, sizeof(double) * (hi - lo));
    }
}

/* Work arrays of one extended pencil of the fluid sweep (index m + GF for m
 * in [-GF, n + GF)). */
typedef struct {
    double *u, *b, *r, *l, *ph1, *uh, *rh, *lh, *sr, *sl, *ph2;
} fluid_work;

static void fluid_work_alloc(fluid_work* w, int W)
{
    w->u = malloc(sizeof(double) * 5 * W);
    w->b = malloc(sizeof(double) * 3 * W);
    w->r = malloc(sizeof(double) * 5 * W);
    w->l = malloc(sizeof(double) * 5 * W);
    w->ph1 = malloc(sizeof(double) * 5 * W);
    w->uh = malloc(sizeof(double) * 5 * W);
    w->rh = malloc(sizeof(double) * 5 * W);
    w->lh = malloc(sizeof(double) * 5 * W);
    w->sr = malloc(sizeof(double) * 5 * W);
    w->sl = malloc(sizeof(double) * 5 * W);
    w->ph2 = malloc(sizeof(double) * 5 * W);
}

static void fluid_work_free(fluid_work* w)
{
    free(w->u); free(w->b); free(w->r); free(w->l); free(w->ph1); free(w->uh);
    free(w->rh); free(w->lh); free(w->sr); free(w->sl); free(w->ph2);
}

/* fluid_d on the d-pencil with transverse coordinates (ae, af). */
static void fluid_pencil(const orc_grid* g, const double* in, double* out, int d, double dt, int ae, int af,
                         fluid_work* w)
{
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    const int n = g->n[d];
    const long N = ncell(g);
    double *u = w->u, *b = w->b, *r = w->r, *l = w->l, *ph1 = w->ph1, *uh = w->uh;
    double *rh = w->rh, *lh = w->lh, *sr = w->sr, *sl = w->sl, *ph2 = w->ph2;
#define AT(a, m) ((a) + 5 * ((m) + GF))

    const int mom[3] = {MX + d, MX + e, MX + f};
    const int bf[3] = {BX + d, BX + e, BX + f};
    const int ax[3] = {d, e, f};

    /* load the extended pencil: conserved u (normal momentum second) and
     * the cell-centred field, the mean of the two faces (Alg. 1 step 3). */
    for (int m = -GF; m < n + GF; m++) {
        int c[3];
        c[d] = m; c[e] = ae; c[f] = af;
        long i0 = lin(g, c);
        double* uu = AT(u, m);
        uu[0] = fld(g, in, RHO)[i0];
        uu[1] = fld(g, in, mom[0])[i0];
        uu[2] = fld(g, in, mom[1])[i0];
        uu[3] = fld(g, in, mom[2])[i0];
        uu[4] = fld(g, in, EN)[i0];
        double* bb = b + 3 * (m + GF);
        for (int q = 0; q < 3; q++) {
            int cp[3] = {c[0], c[1], c[2]};
            cp[ax[q]] += 1;
            bb[q] = 0.5 * (fld(g, in, bf[q])[i0] + fld(g, in, bf[q])[lin(g, cp)]);
        }
    }
    /* stage 1: first-order upwind fluxes from the movers of u^t
     * (eq. Delta_u_half): F_{m+1/2} = r_m - l_{m+1}. */
    for (int m = -GF; m < n + GF; m++) movers(AT(u, m), b + 3 * (m + GF), g->gamma, AT(r, m), AT(l, m));
    for (int m = -GF; m < n + GF - 1; m++)
        for (int q = 0; q < 5; q++) AT(ph1, m)[q] = AT(r, m)[q] - AT(l, m + 1)[q];
    for (int m = -GF + 1; m < n + GF - 1; m++)
        for (int q = 0; q < 5; q++)
            AT(uh, m)[q] = AT(u, m)[q] - (dt / 2.0) * (AT(ph1, m)[q] - AT(ph1, m - 1)[q]);
    /* stage 2: movers of u^{t+dt/2} (Alg. 1 step 7, same field), MUSCL
     * corrections with the van Leer limiter, and the full update from
     * u^t (eq. Delta_u_full). */
    for (int m = -GF + 1; m < n + GF - 1; m++)
        movers(AT(uh, m), b + 3 * (m + GF), g->gamma, AT(rh, m), AT(lh, m));
    for (int m = -GF + 2; m < n + GF - 2; m++)
        for (int q = 0; q < 5; q++) {
            AT(sr, m)[q] = slope(AT(rh, m - 1)[q], AT(rh, m)[q], AT(rh, m + 1)[q]);
            AT(sl, m)[q] = slope(AT(lh, m - 1)[q], AT(lh, m)[q], AT(lh, m + 1)[q]);
        }
    /* right mover upwinded from cell m, left mover from cell m+1 */
    for (int m = -1; m < n; m++)
        for (int q = 0; q < 5; q++)
            AT(ph2, m)[q] = (AT(rh, m)[q] + AT(sr, m)[q]) - (AT(lh, m + 1)[q] - AT(sl, m + 1)[q]);
    for (int m = 0; m < n; m++) {
        int c[3];
        c[d] = m; c[e] = ae; c[f] = af;
        long i0 = lin(g, c);
        const int dst[5] = {RHO, mom[0], mom[1], mom[2], EN};
        for (int q = 0; q < 5; q++)
            out[(long)dst[q] * N + i0] = AT(u, m)[q] - dt * (AT(ph2, m)[q] - AT(ph2, m - 1)[q]);
    }
#undef AT
}

void orc_fluid_sweep(const orc_grid* g, const double* in, double* out, int d, double dt)
{
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    const long N = ncell(g);
    const long npen = (long)g->n[e] * g->n[f];
    copy_state(g, in, out);
#pragma omp parallel
    {
        fluid_work w;
        fluid_work_alloc(&w, g->n[d] + 2 * GF);
#pragma omp for schedule(static)
        for (long p = 0; p < npen; p++)
            fluid_pencil(g, in, out, d, dt, (int)(p % g->n[e]), (int)(p / g->n[e]), &w);
        fluid_work_free(&w);
    }
}

/*
 * EMF of one transverse face component k (k != d) along the d-pencil whose
 * transverse coordinates are those of c0 (c0[k] may lie one past the grid; the
 * EMF there is computed from boundary-mapped primary state).
 * On return G[m + 1] for m in [-1, n) is the limited upwind EMF v_d B_k at the
 * edge between faces m and m+1 of the pencil (Sec. 3, eq. averaging_x and
 * eq. first_flux; Alg. 2 steps 4-8).
 */
static void emf_pencil(const orc_grid* g, const double* s, int d, int k, const int c0[3], double dt, double* G)
{
    const int n = g->n[d];
    const int W = n + 2 * GB;
    double* vhat = malloc(sizeof(double) * W);
    double* bk = malloc(sizeof(double) * W);
    double* v = malloc(sizeof(double) * W);
    double* q = malloc(sizeof(double) * W);
    double* vh = malloc(sizeof(double) * W);
    double* g1 = malloc(sizeof(double) * W);
    double* bh = malloc(sizeof(double) * W);
    double* qh = malloc(sizeof(double) * W);
    double* sq = malloc(sizeof(double) * W);
#define X(a, m) ((a)[(m) + GB])
    const double* rho = fld(g, s, RHO);
    const double* md = fld(g, s, MX + d);
    const double* B = fld(g, s, BX + k);

    /* fluid velocity along d on the k-face: mass-weighted mean of the two
     * cells that share the face (Alg. 2 step 4). */
    for (int m = -GB; m < n + GB; m++) {
        int c[3] = {c0[0], c0[1], c0[2]};
        c[d] = m;
        int cl[3] = {c[0], c[1], c[2]};
        cl[k] -= 1;
        long i0 = lin(g, c), il = lin(g, cl);
        X(vhat, m) = (md[il] + md[i0]) / (rho[il] + rho[i0]);
        X(bk, m) = B[i0];
    }
    /* 1-2-1 smoothing along d (eq. averaging_x) */
    for (int m = -GB + 1; m < n + GB - 1; m++) X(v, m) = 0.25 * (X(vhat, m - 1) + 2.0 * X(vhat, m) + X(vhat, m + 1));
    for (int m = -GB + 1; m < n + GB - 1; m++) X(q, m) = X(v, m) * X(bk, m);
    /* edge velocity and first-order upwind EMF (eq. first_flux) */
    for (int m = -GB + 1; m < n + GB - 2; m++) {
        X(vh, m) = 0.5 * (X(v, m) + X(v, m + 1));
        X(g1, m) = X(vh, m) > 0.0 ? X(q, m) : X(q, m + 1);
    }
    /* half step of the advected component */
    for (int m = -GB + 2; m < n + GB - 2; m++) X(bh, m) = X(bk, m) - (dt / 2.0) * (X(g1, m) - X(g1, m - 1));
    for (int m = -GB + 2; m < n + GB - 2; m++) X(qh, m) = X(v, m) * X(bh, m);
    for (int m = -GB + 3; m < n + GB - 3; m++) X(sq, m) = slope(X(qh, m - 1), X(qh, m), X(qh, m + 1));
    /* second-order upwind EMF from the half-step field */
    for (int m = -1; m < n; m++)
        G[m + 1] = X(vh, m) > 0.0 ? X(qh, m) + X(sq, m) : X(qh, m + 1) - X(sq, m + 1);
#undef X
    free(vhat); free(bk); free(v); free(q); free(vh); free(g1); free(bh); free(qh); free(sq);
}

/* B_{e->d} and B_{f->d} on the d-pencil with transverse coordinates (ae, af);
 * G holds four EMF arrays of n + 1 values. */
static void ct_pencil(const orc_grid* g, const double* in, double* out, int d, double dt, int ae, int af,
                      double* G)
{
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    const int n = g->n[d];
    const long N = ncell(g);
    double* Ge0 = G;
    double* Ge1 = G + (n + 1);
    double* Gf0 = G + 2 * (n + 1);
    double* Gf1 = G + 3 * (n + 1);
    const double* Bd = fld(g, in, BX + d);
    const double* Be = fld(g, in, BX + e);
    const double* Bf = fld(g, in, BX + f);
    double* oBd = out + (long)(BX + d) * N;
    double* oBe = out + (long)(BX + e) * N;
    double* oBf = out + (long)(BX + f) * N;

    int c0[3];
    c0[d] = 0; c0[e] = ae; c0[f] = af;
    int c1[3] = {c0[0], c0[1], c0[2]};
    c1[e] += 1;
    int c2[3] = {c0[0], c0[1], c0[2]};
    c2[f] += 1;
    /* B_{e->d} and B_{f->d}: both read the same (frozen) fluid state */
    emf_pencil(g, in, d, e, c0, dt, Ge0);
    emf_pencil(g, in, d, e, c1, dt, Ge1);
    emf_pencil(g, in, d, f, c0, dt, Gf0);
    emf_pencil(g, in, d, f, c2, dt, Gf1);
    for (int m = 0; m < n; m++) {
        int c[3];
        c[d] = m; c[e] = ae; c[f] = af;
        long i0 = lin(g, c);
        /* advection of the transverse components: -dt d_d(v_d B_k) */
        oBe[i0] = Be[i0] - dt * (Ge0[m + 1] - Ge0[m]);
        oBf[i0] = Bf[i0] - dt * (Gf0[m + 1] - Gf0[m]);
        /* constraint: the same EMFs update B_d on face m (between
         * cells m-1 and m), +dt d_k(v_d B_k); e contribution first. */
        oBd[i0] = (Bd[i0] + dt * (Ge1[m] - Ge0[m])) + dt * (Gf1[m] - Gf0[m]);
    }
}

void orc_ct_sweep(const orc_grid* g, const double* in, double* out, int d, double dt)
{
    const int e = (d + 1) % 3, f = (d + 2) % 3;
    const int n = g->n[d];
    const long N = ncell(g);
    const long npen = (long)g->n[e] * g->n[f];
    copy_state(g, in, out);
#pragma omp parallel
    {
        double* G = malloc(sizeof(double) * 4 * (n + 1));
#pragma omp for schedule(static)
        for (long p = 0; p < npen; p++) ct_pencil(g, in, out, d, dt, (int)(p % g->n[e]), (int)(p / g->n[e]), G);
        free(G);
    }
}

double orc_cmax(const orc_grid* g, const double* s)
{
    double cmax = 0.0;
    int saw_nan = 0;
#pragma omp parallel for schedule(static) reduction(max : cmax) reduction(| : saw_nan)
    for (int k = 0; k < g->n[2]; k++)
        for (int j = 0; j < g->n[1]; j++)
            for (int i = 0; i < g->n[0]; i++) {
                int c[3] = {i, j, k};
                long i0 = lin(g, c);
                double rho = fld(g, s, RHO)[i0];
                double v[3], b[3];
                for (int a = 0; a < 3; a++) {
                    int cp[3] = {i, j, k};
                    cp[a] += 1;
                    v[a] = fld(g, s, MX + a)[i0] / rho;
                    b[a] = 0.5 * (fld(g, s, BX + a)[i0] + fld(g, s, BX + a)[lin(g, cp)]);
                }
                double bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
                double vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
                double p = (g->gamma - 1.0) * (fld(g, s, EN)[i0] - 0.5 * rho * vv - 0.5 * bb);
                /* eq. equat_CFL: largest |v| component plus the fast speed bound */
                double vm = fmax(fabs(v[0]), fmax(fabs(v[1]), fabs(v[2])));
                double cc = vm + sqrt(fabs(g->gamma * p + bb) / rho);
                if (isnan(cc)) saw_nan = 1;
                else if (cc > cmax) cmax = cc;
            }
    return saw_nan ? NAN : cmax;
}

int orc_dt(double cmax, double cfl, double t, double t_stop, double* dt, double* t_new)
{
    /* dt = cfl / c_max; with a stop time the last step is clipped so that
     * t + 2 dt lands exactly on it, after which dt = 0. */
    if (!(cmax > 0.0) || isinf(cmax)) return -4;
    double h = cfl / cmax;
    double tn = t + 2.0 * h;
    if (t_stop >= 0.0) {
        double rem = t_stop - t;
        if (rem <= 0.0) {
            h = 0.0;
            tn = t;
        } else if (2.0 * h >= rem) {
            h = rem / 2.0;
            tn = t_stop;
        }
    }
    *dt = h;
    *t_new = tn;
    return 0;
}

void orc_step_dt(const orc_grid* g, double* s, double dt, long long step)
{
    /* eq. L_sequence: the sweep order rotates (x,y,z) -> (z,x,y) -> (y,z,x);
     * a forward sweep applies L_d = fluid_d, B_{e->d}, B_{f->d} in that order,
     * the reverse sweep the reversed axes with the B updates first. */
    static const int perm[3][3] = {{0, 1, 2}, {2, 0, 1}, {1, 2, 0}};
    const int* p = perm[step % 3];
    long N = ncell(g);
    double* tmp = malloc(sizeof(double) * NF * N);
    for (int a = 0; a < 3; a++) {
        orc_fluid_sweep(g, s, tmp, p[a], dt);
        orc_ct_sweep(g, tmp, s, p[a], dt);
    }
    for (int a = 2; a >= 0; a--) {
        orc_ct_sweep(g, s, tmp, p[a], dt);
        orc_fluid_sweep(g, tmp, s, p[a], dt);
    }
    free(tmp);
}

int orc_step(const orc_grid* g, double* s, double cfl, double t_stop, double* t, long long* step)
{
    double dt, tn;
    int rc = orc_dt(orc_cmax(g, s), cfl, *t, t_stop, &dt, &tn);
    if (rc) return rc;
    orc_step_dt(g, s, dt, *step);
    *t = tn;
    *step += 1;
    return 0;
}

double orc_divb_max(const orc_grid* g, const double* s)
{
    double mx = 0.0;
#pragma omp parallel for schedule(static) reduction(max : mx)
    for (int k = 0; k < g->n[2]; k++)
        for (int j = 0; j < g->n[1]; j++)
            for (int i = 0; i < g->n[0]; i++) {
                int c[3] = {i, j, k};
                int skip = 0;
                if (g->bc != 0)
                    for (int a = 0; a < 3; a++)
                        if (g->n[a] > 1 && c[a] == g->n[a] - 1) skip = 1;
                if (skip) continue;
                long i0 = lin(g, c);
                double div = 0.0;
                for (int a = 0; a < 3; a++) {
                    int cp[3] = {i, j, k};
                    cp[a] += 1;
                    div += fld(g, s, BX + a)[lin(g, cp)] - fld(g, s, BX + a)[i0];
                }
                if (fabs(div) > mx) mx = fabs(div);
            }
    return mx;
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

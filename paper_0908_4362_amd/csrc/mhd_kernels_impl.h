// HIP kernels (gfx950) of one time step of the relaxing-TVD + constrained-
// transport ideal-MHD scheme (Wong et al., Sec. 3 and Sec. 4.3).
//
// Data layout: conserved fields u = (rho, m_x, m_y, m_z, E) and face fields
// b = (B_x, B_y, B_z), each field x-fastest with N = nx*ny*nz cells; B_d(c)
// sits on the lower d-face of cell c (eq. equat_b). Every sweep is
// out-of-place (ping-pong buffers), so no workgroup ever reads a value that
// another workgroup of the same launch writes.
//
// Boundaries: every read beyond the grid goes through the per-axis index map
// (periodic wrap or outflow clamp) of the primary state; derived quantities
// beyond the edge are recomputed from mapped primary values, never wrapped.
//
// Sweeps along y and z march through each pencil: a thread owns one x column
// (64 consecutive x per wavefront, so every load and store is coalesced) and
// walks along the sweep axis keeping the stencil window in registers; a pencil
// is cut into chunks that re-run a short warm-up. Sweeps along x hold the
// cells of a row in the lanes of a wavefront and exchange stencil neighbours
// with cross-lane shuffles: a whole periodic row per wavefront (lane-row form,
// K cells per lane), a whole row per workgroup (row form, one cell per lane,
// wavefront ends exchanged through LDS), or 64-cell segments with halo lanes
// (wavefront form).
//
// Cache policy: on states larger than the memory-side last-level cache the
// sweeps write their outputs and read the values no other thread reads with
// non-temporal accesses (put, ld_own); smaller states keep plain ones.
#pragma once
#include <algorithm>
#include <type_traits>
#include <utility>

#include "mhd_internal.h"

namespace mhd {
namespace {

// FP64 instantiations are compiled without FMA contraction and evaluate every
// expression in the same order, with the same divisions, as the CPU oracle,
// so the double-precision path reproduces it bit for bit (the upwind choice of
// the field update is discontinuous at exact ties, which symmetric problems
// produce, so only identical arithmetic makes both take the same branch).
// FP32 instantiations use FMA within an expression and one reciprocal of rho
// per cell.
template <typename T>
constexpr bool kExact = std::is_same<T, double>::value;

// Output stores of the sweeps: non-temporal (`nt`, the written line is not
// kept in the caches) or plain, as the launch chooses (nt_policy). Measured at
// 256^3 against plain stores: FP32 step 1.731 -> 1.691 ms, FP64 3.388 ->
// 3.352 ms (field update along x -6 %, field marches -1 to -2 %, fused sweeps
// -1 %, the fluid y march +3 %); results are the same bits either way.
template <bool NT, typename T>
__device__ __forceinline__ void put(T* p, T v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Loads of values that no other thread of the sweep reads follow the same
// policy: the conserved fields of a fluid update's own cell (256^3 step FP64
// 3.353 -> 3.307 ms, FP32 1.677 -> 1.646 ms with non-temporal loads), the old
// B_d of a march's own cell and a row's own x face field (a further -0.8 % /
// -0.5 %).
template <bool NT, typename T>
__device__ __forceinline__ T ld_own(const T* p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// Division. FP64 quotients must be the correctly rounded ones the oracle
// gets. The compiler's IEEE division is a Newton-Raphson refinement of the
// hardware reciprocal followed by a residual correction (Markstein's method),
// wrapped in range scaling (v_div_scale / v_div_fmas / v_div_fixup) that only
// acts when an operand or the quotient is near the edge of the exponent range
// or not finite. The helpers below run the same refinement without that
// wrapping, so for normal-range operands (every state of a physical run) they
// give the same bits in 8 instructions instead of 11, and a reciprocal that
// several quotients share (the divisions by rho of one cell) is refined once.
// Outside that range (|n| below about 1e-292, a subnormal or zero divisor)
// a quotient may differ from IEEE division in its last bit or be non-finite.
struct Recip64 {
    double y;    // refined reciprocal of d
    double nd;   // -d
};

__device__ __forceinline__ Recip64 recip64(double d)
{
    const double nd = -d;
    const double y0 = __builtin_amdgcn_rcp(d);
    const double e0 = __builtin_fma(nd, y0, 1.0);
    const double y1 = __builtin_fma(y0, e0, y0);
    const double e1 = __builtin_fma(nd, y1, 1.0);
    return {__builtin_fma(y1, e1, y1), nd};
}

__device__ __forceinline__ double div64(double n, const Recip64& r)
{
    const double q = n * r.y;
    const double rem = __builtin_fma(r.nd, q, n);
    return __builtin_fma(rem, r.y, q);
}

// n / d: correctly rounded (normal range) in FP64; in FP32 the hardware
// reciprocal (1 ulp) times n.
template <typename T>
__device__ __forceinline__ T qdiv(T n, T d)
{
    if constexpr (kExact<T>)
        return div64(n, recip64(d));
    else
        return n * __builtin_amdgcn_rcpf(d);
}

// Square root: IEEE in FP64 (the oracle's), the hardware one (1 ulp) in FP32.
template <typename T>
__device__ __forceinline__ T qsqrt(T x)
{
    if constexpr (kExact<T>)
        return sqrt(x);
    else
        return __builtin_amdgcn_sqrtf(x);
}

constexpr int GF = 3;  // ghost depth of the fluid sweep
constexpr int GB = 4;  // ghost depth of the field (CT) sweep

__device__ __forceinline__ int wrap_idx(int i, int n, int bc)
{
    if ((unsigned)i < (unsigned)n) return i;
    if (bc == 0) {
        // one period away covers every ghost unless the grid is shorter
        // than the stencil's reach
        const int r = i < 0 ? i + n : i - n;
        if ((unsigned)r < (unsigned)n) return r;
        const int m = i % n;
        return m < 0 ? m + n : m;
    }
    return i < 0 ? 0 : n - 1;
}

// van Leer limiter (eq. limiter) of the half-differences a/2 and b/2 of a
// stencil, evaluated from the full differences a and b: zero when they differ
// in sign, else 2 (a/2)(b/2) / (a/2 + b/2). Halving is exact, so the product
// and the sum are the rounded ab and a + b scaled by 1/4 and 1/2, and the
// quotient is the rounded ab / (a + b): the same bits, three multiplies fewer,
// whenever ab / 4 and (a + b) / 2 stay in the normal range.
template <typename T>
__device__ __forceinline__ T vanleer_half(T a, T b)
{
    const T ab = a * b;
    return ab > T(0) ? qdiv(ab, a + b) : T(0);
}

// CFL speed of one cell, eq. equat_CFL: largest |v| component plus
// sqrt(|gamma p + B^2| / rho); b is the centred field. FP64 follows the
// oracle's expression order.
template <typename T>
__device__ __forceinline__ T cfl_speed(T rho, T mx, T my, T mz, T en, T bx, T by, T bz, T gamma)
{
    // no contraction: every kernel that evaluates it (the c_max pass, the
    // fluid sweeps that store c_max slots) must get the same bits, so that a
    // run resumed from a stored state takes the same dt
#pragma clang fp contract(off)
    const T bb = bx * bx + by * by + bz * bz;
    if constexpr (kExact<T>) {
        const Recip64 ri = recip64(rho);
        const T vx = div64(mx, ri), vy = div64(my, ri), vz = div64(mz, ri);
        const T vv = vx * vx + vy * vy + vz * vz;
        const T p = (gamma - T(1)) * (en - T(0.5) * rho * vv - T(0.5) * bb);
        const T vm = fmax(fabs(vx), fmax(fabs(vy), fabs(vz)));
        return vm + sqrt(div64(fabs(gamma * p + bb), ri));
    } else {
        const T rinv = __builtin_amdgcn_rcpf(rho);
        const T vx = mx * rinv, vy = my * rinv, vz = mz * rinv;
        const T ke = T(0.5) * (mx * vx + my * vy + mz * vz);
        const T p = (gamma - T(1)) * (en - ke - T(0.5) * bb);
        const T vm = fmax(fabs(vx), fmax(fabs(vy), fabs(vz)));
        return vm + qsqrt(fabs(gamma * p + bb) * rinv);
    }
}

// Ordered bit pattern of a non-negative value (NaN is mapped to the canonical
// positive NaN, which sorts above +inf, so it propagates through a max).
template <typename T>
__device__ __forceinline__ unsigned long long speed_bits(T c)
{
    double d = (double)c;
    if (d != d) d = __builtin_nan("");
    return (unsigned long long)__double_as_longlong(d);
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Max over a block of BS threads (linear id tid); valid in thread 0.
template <int BS>
__device__ __forceinline__ unsigned long long block_max_u64(unsigned long long v, int tid)
{
    __shared__ unsigned long long part[BS / 64];
    v = wave_max_u64(v);
    if ((tid & 63) == 0) part[tid >> 6] = v;
    __syncthreads();
    if (tid < 64) {
        v = tid < BS / 64 ? part[tid] : 0ull;
        v = wave_max_u64(v);
    }
    return v;
}

// Grid-wide max, first level: every block stores its maximum in its own slot
// of a parts array (plain stores, no atomics); a one-block finisher reduces
// the parts.
template <int BS>
__device__ __forceinline__ void block_max_to_part(unsigned long long v, int tid, unsigned long long* slot)
{
    v = block_max_u64<BS>(v, tid);
    if (tid == 0) *slot = v;
}

// Time-step rule (Sec. 4.2, eq. equat_CFL): dt = cfl / c_max, clipped so that
// t + 2 dt lands exactly on the stop time, after which dt = 0; a NaN, infinite
// or non-positive c_max latches the non-finite status.
__device__ __forceinline__ void apply_dt_rule(Ctl* ctl, double cfl)
{
    const double cmax = ctl->cmax;
    double dt = 0.0, t = ctl->t;
    if (ctl->status == 0) {
        if (!(cmax > 0.0) || cmax > 1.7976931348623157e308) {
            ctl->status = -4;
        } else {
            double h = cfl / cmax;
            double tn = t + 2.0 * h;
            const double ts = ctl->t_stop;
            if (ts >= 0.0) {
                const double rem = ts - t;
                if (rem <= 0.0) {
                    h = 0.0;
                    tn = t;
                } else if (2.0 * h >= rem) {
                    h = rem / 2.0;
                    tn = ts;
                }
            }
            dt = h;
            t = tn;
        }
    }
    ctl->dt = dt;
    ctl->t = t;
}

// Movers r = (c u + F)/2 and l = (c u - F)/2 of eq. lr (times c) for a cell
// with conserved u (normal momentum second) and centred field b (normal
// first); F is eq. flux rotated to the sweep axis, c = |v_n| + sqrt(|gamma p +
// B^2| / rho) the per-cell freezing speed.
template <typename T>
__device__ __forceinline__ void movers(const T* u, const T* b, T gamma, T* r, T* l)
{
    T F[5], c;
    if constexpr (kExact<T>) {
        const T rho = u[0];
        const Recip64 ri = recip64(rho);
        const T vn = div64(u[1], ri), v1 = div64(u[2], ri), v2 = div64(u[3], ri);
        const T bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
        const T vv = vn * vn + v1 * v1 + v2 * v2;
        const T p = (gamma - T(1)) * (u[4] - T(0.5) * rho * vv - T(0.5) * bb);
        const T ps = p + T(0.5) * bb;
        const T bv = b[0] * vn + b[1] * v1 + b[2] * v2;
        F[0] = u[1];
        F[1] = u[1] * vn + ps - b[0] * b[0];
        F[2] = u[2] * vn - b[0] * b[1];
        F[3] = u[3] * vn - b[0] * b[2];
        F[4] = (u[4] + ps) * vn - b[0] * bv;
        c = fabs(vn) + sqrt(div64(fabs(gamma * p + bb), ri));
    } else {
        const T rinv = __builtin_amdgcn_rcpf(u[0]);
        const T vn = u[1] * rinv, v1 = u[2] * rinv, v2 = u[3] * rinv;
        const T bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
        const T ke = T(0.5) * (u[1] * vn + u[2] * v1 + u[3] * v2);
        const T p = (gamma - T(1)) * (u[4] - ke - T(0.5) * bb);
        const T ps = p + T(0.5) * bb;
        const T bv = b[0] * vn + b[1] * v1 + b[2] * v2;
        F[0] = u[1];
        F[1] = u[1] * vn + ps - b[0] * b[0];
        F[2] = u[2] * vn - b[0] * b[1];
        F[3] = u[3] * vn - b[0] * b[2];
        F[4] = (u[4] + ps) * vn - b[0] * bv;
        c = fabs(vn) + qsqrt(fabs(gamma * p + bb) * rinv);
    }
#pragma unroll
    for (int q = 0; q < 5; q++) {
        r[q] = T(0.5) * (c * u[q] + F[q]);
        l[q] = T(0.5) * (c * u[q] - F[q]);
    }
}

// ---------------------------------------------------------------------------
// Register pipeline of the fluid sweep. push() consumes the conserved state
// and centred field of the head cell h and returns the updated state of cell
// h - 3 (valid once the window is full).
template <typename T>
struct FluidPipe {
    T r1[5];          // r at h-1
    T f1[5];          // first-order flux at (h-1) - 1/2
    T u1[5], u2[5], u3[5];  // conserved state at h-1, h-2, h-3
    T b1[3], b2[3], b3[3];  // centred field at h-1, h-2, h-3
    T rp2[5], rp3[5], lp2[5], lp3[5];  // movers of u^{t+dt/2} at h-2, h-3
    T R3[5];          // limited right mover at h-3
    T f2[5];          // second-order flux at (h-3) - 1/2

    __device__ __forceinline__ void clear()
    {
#pragma unroll
        for (int q = 0; q < 5; q++) {
            r1[q] = f1[q] = u1[q] = u2[q] = u3[q] = T(0);
            rp2[q] = rp3[q] = lp2[q] = lp3[q] = R3[q] = f2[q] = T(0);
        }
        b1[0] = b1[1] = b1[2] = T(0);
        b2[0] = b2[1] = b2[2] = T(0);
        b3[0] = b3[1] = b3[2] = T(0);
    }

    __device__ __forceinline__ void push(const T* uh, const T* bh, T gamma, T dt, T* unew)
    {
        T rh[5], lh[5];
        movers(uh, bh, gamma, rh, lh);
        // stage 1 (eq. Delta_u_half): first-order upwind flux r_{h-1} - l_h at
        // face h - 1/2, half step of cell h-1
        T fh[5], uhalf[5];
#pragma unroll
        for (int q = 0; q < 5; q++) {
            fh[q] = r1[q] - lh[q];
            uhalf[q] = u1[q] - (dt * T(0.5)) * (fh[q] - f1[q]);
        }
        // stage 2 (Alg. 1 step 7, eq. Delta_u_full): movers of u^{t+dt/2} at
        // h-1 with the same field, van Leer limited slopes at h-2
        T rp1[5], lp1[5];
        movers(uhalf, b1, gamma, rp1, lp1);
        T R2[5];
#pragma unroll
        for (int q = 0; q < 5; q++) {
            const T sr = vanleer_half(rp2[q] - rp3[q], rp1[q] - rp2[q]);
            const T sl = vanleer_half(lp2[q] - lp3[q], lp1[q] - lp2[q]);
            R2[q] = rp2[q] + sr;
            const T L2 = lp2[q] - sl;
            // flux at (h-3) + 1/2: right mover from h-3, left mover from h-2
            const T f = R3[q] - L2;
            unew[q] = u3[q] - dt * (f - f2[q]);
            f2[q] = f;
        }
#pragma unroll
        for (int q = 0; q < 5; q++) {
            R3[q] = R2[q];
            rp3[q] = rp2[q];
            rp2[q] = rp1[q];
            lp3[q] = lp2[q];
            lp2[q] = lp1[q];
            f1[q] = fh[q];
            r1[q] = rh[q];
            u3[q] = u2[q];
            u2[q] = u1[q];
            u1[q] = uh[q];
        }
#pragma unroll
        for (int q = 0; q < 3; q++) {
            b3[q] = b2[q];
            b2[q] = b1[q];
            b1[q] = bh[q];
        }
    }
};

// Register pipeline of one EMF along the sweep (Alg. 2 steps 4-8). push()
// consumes the raw face velocity and face field of head h and returns the
// limited upwind EMF at edge (h-4) + 1/2.
template <typename T>
struct EmfPipe {
    T vh1, vh2;       // raw face velocity at h-1, h-2
    T v2;             // smoothed velocity at h-2
    T B1, B2, B3, B4; // face field at h-1 .. h-4
    T g3;             // first-order EMF at edge (h-3) + 1/2
    T qh3, qh4;       // v B^{t+dt/2} at h-3, h-4
    T s4;             // limited slope at h-4
    T e3, e4;         // edge velocity at (h-3) + 1/2, (h-4) + 1/2
    T G5;             // EMF at edge (h-5) + 1/2

    __device__ __forceinline__ void clear()
    {
        vh1 = vh2 = v2 = B1 = B2 = B3 = B4 = g3 = qh3 = qh4 = s4 = e3 = e4 = G5 = T(0);
    }

    __device__ __forceinline__ T push(T vhat, T Bh, T dt)
    {
        // 1-2-1 smoothing along the sweep (eq. averaging_x) -> v at h-1
        const T v1 = T(0.25) * (vh2 + T(2) * vh1 + vhat);
        const T q1 = v1 * B1;
        const T q2 = v2 * B2;
        // edge velocity and first-order upwind EMF at (h-2) + 1/2 (eq. first_flux)
        const T e2 = T(0.5) * (v2 + v1);
        const T g2 = e2 > T(0) ? q2 : q1;
        // half step of the advected component at h-2
        const T bh2 = B2 - (dt * T(0.5)) * (g2 - g3);
        const T qh2 = v2 * bh2;
        // limited slope at h-3 and second-order EMF at (h-4) + 1/2
        const T s3 = vanleer_half(qh3 - qh4, qh2 - qh3);
        const T G4 = e4 > T(0) ? qh4 + s4 : qh3 - s3;
        e4 = e3;
        e3 = e2;
        s4 = s3;
        qh4 = qh3;
        qh3 = qh2;
        g3 = g2;
        B4 = B3;
        B3 = B2;
        B2 = B1;
        B1 = Bh;
        v2 = v1;
        vh2 = vh1;
        vh1 = vhat;
        return G4;
    }
};

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// fluid_d for d = y (D = 1) or z (D = 2): marching kernel.
// Block (64, MW): lanes along x, MW wavefronts along the remaining axis TA;
// 1D grid of ntx * ntg * nch tiles (x tiles fastest, then TA groups, then
// chunks along d). With CFL the kernel also reduces c_max of the state it
// writes (the last sweep of a step), so the next step needs no extra pass.
constexpr int MW = 4;   // wavefronts per marching workgroup

// Wavefronts per marching launch, measured best on 256^3: 2048 (chunks of 128
// cells, half the warm-up of 64-cell chunks) except for the FP32 field sweep,
// which at occupancy 4 needs 4096 to fill the device.
constexpr long long kFluidMarchWaves = 2048;
template <typename T>
constexpr long long kCtMarchWaves = kExact<T> ? 2048 : 4096;

struct MarchTile {
    int i, tc, o0, o1;
    bool active;
};

// Wavefronts of a marching workgroup placed side by side along x: a y sweep's
// transverse axis is z, whose neighbouring planes lie far apart in memory, so
// its MW wavefronts go along x as far as the row holds them (each then reads
// one contiguous stretch of a row; 3-4 % faster at 256^3) and the rest along
// z. The FP64 field sweep keeps them along z (xwide false): it reads the -z
// and +z neighbours of rho and m_d, which a workgroup along z shares (2 %
// faster that way). A z sweep's transverse neighbours are adjacent rows, so
// its wavefronts stay along y. Either way a transverse axis shorter than the
// workgroup (nt = 1 on a plane) would leave wavefronts without a pencil, so
// the workgroup then puts along x as many as the transverse axis cannot take.
__host__ __device__ inline int march_wx(int axis, int nx, int nt, bool xwide)
{
    int wx = 1;
    if (axis == 1 && xwide)
        while (wx < MW && 128 * wx <= nx) wx *= 2;
    while (wx < MW && nt * wx < MW) wx *= 2;
    return wx;
}

// xwide of the fluid (CT = false) and field (CT = true) sweeps.
template <typename T, bool CT>
constexpr bool kMarchXWide = !(CT && kExact<T>);

// Rows that are not a multiple of 64 cells would leave lanes of their last
// wavefront idle (a 96-cell row keeps 96 of 128 lanes busy, a 32-cell row
// half): there the lanes of a marching launch take consecutive positions of
// the flattened (x, TA) plane instead, x fastest and running on into the next
// transverse row (packed layout), so every lane but those past the plane's
// end has a pencil. A pencil's arithmetic does not depend on which lane runs
// it, so the layout never changes a result.
__host__ __device__ inline bool march_packed(int nx) { return nx % 64 != 0; }

template <int D, bool XWIDE>
__device__ __forceinline__ MarchTile march_tile(const Grid& g, int chunk, unsigned lb)
{
    constexpr int TA = (D == 1) ? 2 : 1;
    const int nx = g.n[0], nd = g.n[D], nt = g.n[TA];
    if (march_packed(nx)) {
        const long long P = (long long)nx * nt;
        const unsigned ntp = (unsigned)((P + 64 * MW - 1) / (64 * MW));
        const unsigned pt = lb % ntp, ch = lb / ntp;
        const long long c = (long long)pt * (64 * MW) + threadIdx.y * 64 + threadIdx.x;
        MarchTile m;
        m.i = (int)(c % nx);
        m.tc = (int)(c / nx);
        m.o0 = ch * chunk;
        m.o1 = min(m.o0 + chunk, nd);
        m.active = c < P && m.o0 < m.o1;
        return m;
    }
    const unsigned wx = (unsigned)march_wx(D, nx, nt, XWIDE), wt = MW / wx;
    const unsigned ntx = (nx + 64 * wx - 1) / (64 * wx), ntg = (nt + wt - 1) / wt;
    const unsigned xt = lb % ntx, rest = lb / ntx;
    const unsigned tg = rest % ntg, ch = rest / ntg;
    MarchTile m;
    m.i = (xt * wx + threadIdx.y % wx) * 64 + threadIdx.x;
    m.tc = tg * wt + threadIdx.y / wx;
    m.o0 = ch * chunk;
    m.o1 = min(m.o0 + chunk, nd);
    m.active = m.i < nx && m.tc < nt && m.o0 < m.o1;
    return m;
}

// Marching kernels: each thread walks its pencil cell by cell. The global
// loads of cell h + 1 are issued before the arithmetic of cell h, so their
// latency overlaps it (the compiler does not pipeline the loop by itself).
// Neighbour values across x come from the adjacent lanes' cache lines, those
// across the other transverse axis TA from the neighbouring pencil, read
// directly (an LDS exchange between the wavefronts of a workgroup costs a
// barrier per cell and measured slower).
template <typename T>
struct FluidLoad {
    T u[5];
    T bd1;        // B_d on the upper d-face
    T bt0, bt1;   // transverse face field (axis TA) on the lower / upper face
    T bx0, bx1;   // x face field on the lower / upper face
};

template <typename T, int D, bool CFL, bool NT = true>
__device__ __forceinline__ void fluid_march_body(const T* __restrict__ uin, T* __restrict__ uout,
                                                 const T* __restrict__ bf, const Grid& g, T gamma,
                                                 const Ctl* __restrict__ ctl, double dt_arg, int chunk, unsigned lb,
                                                 unsigned long long* __restrict__ part)
{
    constexpr int E = (D + 1) % 3, F = (D + 2) % 3;
    constexpr int TA = (D == 1) ? 2 : 1;
    // the transverse axis TA is E for a sweep along y and F for a sweep along z
    constexpr bool T_IS_E = (E == TA);
    const MarchTile mt = march_tile<D, kMarchXWide<T, false>>(g, chunk, lb);
    const int nx = g.n[0], nd = g.n[D], nt = g.n[TA];
    const int o0 = mt.o0, o1 = mt.o1;
    const int i = wrap_idx(mt.i, nx, g.bc), tc = wrap_idx(mt.tc, nt, g.bc);
    const bool active = mt.active;
    const long long N = g.N;
    const long long sd = (D == 1) ? (long long)nx : (long long)nx * g.n[1];
    const long long st = (TA == 1) ? (long long)nx : (long long)nx * g.n[1];
    const long long base = i + tc * st;
    const long long offX = wrap_idx(i + 1, nx, g.bc) - i;
    const long long offT = (long long)(wrap_idx(mt.tc + 1, nt, g.bc) - tc) * st;
    const T* rho = uin;
    const T* mD = uin + (1 + D) * N;
    const T* mE = uin + (1 + E) * N;
    const T* mF = uin + (1 + F) * N;
    const T* en = uin + 4 * N;
    const T* BD = bf + D * N;
    const T* BT = bf + (T_IS_E ? E : F) * N;
    const T* BX = bf + (T_IS_E ? F : E) * N;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;
    unsigned long long best = 0ull;

    auto load = [&](int h, FluidLoad<T>& L) {
        const long long c = base + (long long)wrap_idx(h, nd, g.bc) * sd;
        L.u[0] = ld_own<NT>(&rho[c]);
        L.u[1] = ld_own<NT>(&mD[c]);
        L.u[2] = ld_own<NT>(&mE[c]);
        L.u[3] = ld_own<NT>(&mF[c]);
        L.u[4] = ld_own<NT>(&en[c]);
        L.bd1 = ld_own<NT>(&BD[base + (long long)wrap_idx(h + 1, nd, g.bc) * sd]);
        L.bt0 = BT[c];
        L.bt1 = BT[c + offT];
        L.bx0 = BX[c];
        L.bx1 = BX[c + offX];
    };

    FluidPipe<T> P;
    P.clear();
    T bd_lo = BD[base + (long long)wrap_idx(o0 - GF, nd, g.bc) * sd];
    FluidLoad<T> cur;
    load(o0 - GF, cur);
    for (int h = o0 - GF; h <= o1 + GF - 1; ++h) {
        FluidLoad<T> nxt;
        load(h + 1, nxt);   // one cell past the end is a valid (mapped) cell
        const T bT = T(0.5) * (cur.bt0 + cur.bt1), bX = T(0.5) * (cur.bx0 + cur.bx1);
        T bh[3] = {T(0.5) * (bd_lo + cur.bd1), T_IS_E ? bT : bX, T_IS_E ? bX : bT};
        bd_lo = cur.bd1;
        const T keep[5] = {P.u3[0], P.u3[1], P.u3[2], P.u3[3], P.u3[4]};
        const T bo[3] = {P.b3[0], P.b3[1], P.b3[2]};   // centred field of the output cell
        T un[5];
        P.push(cur.u, bh, gamma, dt, un);
        const int o = h - GF;
        if (active && o >= o0) {
            if (frozen) {
#pragma unroll
                for (int q = 0; q < 5; q++) un[q] = keep[q];
            }
            const long long co = base + (long long)o * sd;
            put<NT>(&uout[co], un[0]);
            put<NT>(&uout[(1 + D) * N + co], un[1]);
            put<NT>(&uout[(1 + E) * N + co], un[2]);
            put<NT>(&uout[(1 + F) * N + co], un[3]);
            put<NT>(&uout[4 * N + co], un[4]);
            if constexpr (CFL) {
                // back to x, y, z order: rotated slot of axis a is (a - D) mod 3
                const T cc = cfl_speed(un[0], un[1 + (3 - D) % 3], un[1 + (4 - D) % 3], un[1 + (5 - D) % 3],
                                       un[4], bo[(3 - D) % 3], bo[(4 - D) % 3], bo[(5 - D) % 3], gamma);
                const unsigned long long bits = speed_bits(cc);
                best = bits > best ? bits : best;
            }
        }
        cur = nxt;
    }
    if constexpr (CFL) block_max_to_part<64 * MW>(best, threadIdx.x + 64 * threadIdx.y, part);
}

// Slot count of a c_max producer of the plain solver, stored for the
// finisher by one thread of the launch.
__device__ __forceinline__ void store_part_count(int* count)
{
    if (blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) *count = (int)gridDim.x;
}

template <typename T, int D, bool CFL, bool NT>
__global__ void __launch_bounds__(64 * MW) fluid_march(const T* __restrict__ uin, T* __restrict__ uout,
                                                       const T* __restrict__ bf, Grid g, T gamma,
                                                       const Ctl* __restrict__ ctl, double dt_arg, int chunk,
                                                       unsigned long long* __restrict__ parts, int* count)
{
    const unsigned lb = blockIdx.x;
    if constexpr (CFL) store_part_count(count);
    fluid_march_body<T, D, CFL, NT>(uin, uout, bf, g, gamma, ctl, dt_arg, chunk, lb, parts + blockIdx.x);
}

// B_{e->d}, B_{f->d} for d = y or z: marching kernel, same launch shape as
// fluid_march. Each thread runs four EMF pipelines: the TA- and x-face pencils
// through its own cells and through the +TA / +x neighbours (their EMFs enter
// the constraint update of B_d).
template <typename T>
struct CtLoad {
    T r0, m0, bt;            // own cell: rho, m_d, TA face field
    T rTm, mTm, rTp, mTp, bt1;   // TA -1 / +1 neighbours
    T rXm, mXm, rXp, mXp, bx0, bx1;
};

template <typename T, int D, bool NT = true>
__device__ __forceinline__ void ct_march_body(const T* __restrict__ uf, const T* __restrict__ bin,
                                              T* __restrict__ bout, const Grid& g, const Ctl* __restrict__ ctl,
                                              double dt_arg, int chunk, unsigned lb)
{
    constexpr int E = (D + 1) % 3, F = (D + 2) % 3;
    constexpr int TA = (D == 1) ? 2 : 1;
    constexpr bool T_IS_E = (E == TA);
    const MarchTile mt = march_tile<D, kMarchXWide<T, true>>(g, chunk, lb);
    const int nx = g.n[0], nd = g.n[D], nt = g.n[TA];
    const int o0 = mt.o0, o1 = mt.o1;
    const int i = wrap_idx(mt.i, nx, g.bc), tc = wrap_idx(mt.tc, nt, g.bc);
    const bool active = mt.active;
    const long long N = g.N;
    const long long sd = (D == 1) ? (long long)nx : (long long)nx * g.n[1];
    const long long st = (TA == 1) ? (long long)nx : (long long)nx * g.n[1];
    const long long base = i + tc * st;
    const long long xp = wrap_idx(i + 1, nx, g.bc) - i;
    const long long xm_ = wrap_idx(i - 1, nx, g.bc) - i;
    const long long lo = (long long)(wrap_idx(mt.tc - 1, nt, g.bc) - tc) * st;
    const long long hi = (long long)(wrap_idx(mt.tc + 1, nt, g.bc) - tc) * st;
    const T* rho = uf;
    const T* md = uf + (1 + D) * N;
    const T* BD = bin + D * N;
    const T* BT = bin + (T_IS_E ? E : F) * N;
    const T* BX = bin + (T_IS_E ? F : E) * N;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;

    auto load = [&](int h, CtLoad<T>& L) {
        const long long c = base + (long long)wrap_idx(h, nd, g.bc) * sd;
        L.r0 = rho[c];
        L.m0 = md[c];
        L.bt = BT[c];
        L.rTm = rho[c + lo];
        L.mTm = md[c + lo];
        L.rTp = rho[c + hi];
        L.mTp = md[c + hi];
        L.bt1 = BT[c + hi];
        L.rXm = rho[c + xm_];
        L.mXm = md[c + xm_];
        L.rXp = rho[c + xp];
        L.mXp = md[c + xp];
        L.bx0 = BX[c];
        L.bx1 = BX[c + xp];
    };

    EmfPipe<T> t0, t1, x0, x1;   // TA-face pencils (own, +TA), x-face pencils (own, +x)
    t0.clear();
    t1.clear();
    x0.clear();
    x1.clear();
    CtLoad<T> cur;
    load(o0 - GB, cur);
    // unrolled so that the window shifts become register renames: 6 times in
    // FP64, 4 in FP32 (the fastest measured; FP64 16-19 % faster than the
    // rolled loop, FP32 3-7 %)
    constexpr int kUnroll = kExact<T> ? 6 : 4;
#pragma unroll kUnroll
    for (int h = o0 - GB; h <= o1 + GB - 1; ++h) {
        CtLoad<T> nxt;
        load(h + 1, nxt);
        const T r0 = cur.r0, m0 = cur.m0;
        const T rTm = cur.rTm, mTm = cur.mTm, rTp = cur.rTp, mTp = cur.mTp, bt1 = cur.bt1;
        // original transverse faces of the output cell h - 4
        const T bto = t0.B4, bxo = x0.B4;
        // face velocity along d on a transverse face: mass-weighted mean of the
        // two cells sharing it (Alg. 2 step 4)
        const T Gt0 = t0.push(qdiv(mTm + m0, rTm + r0), cur.bt, dt);
        const T Gt1 = t1.push(qdiv(m0 + mTp, r0 + rTp), bt1, dt);
        const T Gx0 = x0.push(qdiv(cur.mXm + m0, cur.rXm + r0), cur.bx0, dt);
        const T Gx1 = x1.push(qdiv(m0 + cur.mXp, r0 + cur.rXp), cur.bx1, dt);
        const int o = h - GB;
        if (active && o >= o0) {
            const long long co = base + (long long)o * sd;
            // *.G5 still hold the EMFs at edge o - 1/2 (updated below)
            const T bd = ld_own<NT>(&BD[co]);
            // e is the cyclic successor of d: the constraint adds the e
            // contribution first
            const T Ge0 = T_IS_E ? Gt0 : Gx0, Ge0p = T_IS_E ? t0.G5 : x0.G5, Ge1p = T_IS_E ? t1.G5 : x1.G5;
            const T Gf0 = T_IS_E ? Gx0 : Gt0, Gf0p = T_IS_E ? x0.G5 : t0.G5, Gf1p = T_IS_E ? x1.G5 : t1.G5;
            const T be = T_IS_E ? bto : bxo, bfv = T_IS_E ? bxo : bto;
            // a frozen state (status set) is copied through unchanged
            const T nE = frozen ? be : be - dt * (Ge0 - Ge0p);
            const T nF = frozen ? bfv : bfv - dt * (Gf0 - Gf0p);
            const T nD = frozen ? bd : (bd + dt * (Ge1p - Ge0p)) + dt * (Gf1p - Gf0p);
            put<NT>(&bout[E * N + co], nE);
            put<NT>(&bout[F * N + co], nF);
            put<NT>(&bout[D * N + co], nD);
        }
        t0.G5 = Gt0;
        t1.G5 = Gt1;
        x0.G5 = Gx0;
        x1.G5 = Gx1;
        cur = nxt;
    }
}

// Workgroups go to the 8 XCDs round-robin; this order gives each XCD a
// contiguous range of logical workgroups, so that the marches of transverse
// neighbours (whose rho and m_d each field march reads) share one L2. It cut
// the field marches' time by 2-5 % at 256^3; the fluid and fused marches
// showed no gain and keep the plain order.
__device__ __forceinline__ unsigned xcd_order(unsigned b, unsigned n)
{
    const unsigned x = b % 8u, q = n / 8u, r = n % 8u;
    return x * q + (x < r ? x : r) + b / 8u;
}

template <typename T, int D, bool NT>
__global__ void __launch_bounds__(64 * MW) ct_march(const T* __restrict__ uf, const T* __restrict__ bin,
                                                    T* __restrict__ bout, Grid g, const Ctl* __restrict__ ctl,
                                                    double dt_arg, int chunk)
{
    ct_march_body<T, D, NT>(uf, bin, bout, g, ctl, dt_arg, chunk, xcd_order(blockIdx.x, gridDim.x));
}


// ---------------------------------------------------------------------------
// Reverse L_d for d = y or z (Sec. 4.3: the field update first, then the
// fluid update) in one march, on periodic grids: B_{e->d}, B_{f->d} (Alg. 2)
// followed by fluid_d (Alg. 1) on the field it produced. The four EMF
// pipelines of ct_march run ahead; they yield the new face fields of the
// thread's own cell and of the faces its +TA / +x neighbours own (the faces
// that enter the centred field), and the fluid pipeline of fluid_march
// follows five cells behind, taking rho and m_d from a delay line of the
// values the EMF pipelines loaded. Every value is computed by the same
// expressions as in ct_march and fluid_march, so the result is the one of the
// two launches, bit for bit, with 16 words of traffic per cell instead of
// 8 + 13. Periodic wrapping makes the new field at a ghost position equal to
// the new field of the cell it maps to; with outflow clamping it would not
// (the two launches run there).
constexpr int GCF = GF + GB;   // ghost depth of the fused march (3 + 4)

template <typename T>
struct FusedLoad {
    T bd;              // B_d (old) of the field update's output cell h - 4
    T me, mf, en;      // m_e, m_f, E of the fluid head cell h - 5
};

template <typename T, int D, bool CFL, bool NT = true>
__device__ __forceinline__ void ct_fluid_march_body(const T* __restrict__ uin, T* __restrict__ uout,
                                                    const T* __restrict__ bin, T* __restrict__ bout, const Grid& g,
                                                    T gamma, const Ctl* __restrict__ ctl, double dt_arg, int chunk,
                                                    unsigned lb, unsigned long long* __restrict__ part)
{
    constexpr int E = (D + 1) % 3, F = (D + 2) % 3;
    constexpr int TA = (D == 1) ? 2 : 1;
    constexpr bool T_IS_E = (E == TA);
    const MarchTile mt = march_tile<D, kMarchXWide<T, true>>(g, chunk, lb);
    const int nx = g.n[0], nd = g.n[D], nt = g.n[TA];
    const int o0 = mt.o0, o1 = mt.o1;
    const int i = wrap_idx(mt.i, nx, g.bc), tc = wrap_idx(mt.tc, nt, g.bc);
    const bool active = mt.active;
    const long long N = g.N;
    const long long sd = (D == 1) ? (long long)nx : (long long)nx * g.n[1];
    const long long st = (TA == 1) ? (long long)nx : (long long)nx * g.n[1];
    const long long base = i + tc * st;
    const long long xp = wrap_idx(i + 1, nx, g.bc) - i;
    const long long xm_ = wrap_idx(i - 1, nx, g.bc) - i;
    const long long lo = (long long)(wrap_idx(mt.tc - 1, nt, g.bc) - tc) * st;
    const long long hi = (long long)(wrap_idx(mt.tc + 1, nt, g.bc) - tc) * st;
    const T* rho = uin;
    const T* md = uin + (1 + D) * N;
    const T* mE = uin + (1 + E) * N;
    const T* mF = uin + (1 + F) * N;
    const T* en = uin + 4 * N;
    const T* BD = bin + D * N;
    const T* BT = bin + (T_IS_E ? E : F) * N;
    const T* BX = bin + (T_IS_E ? F : E) * N;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;
    unsigned long long best = 0ull;

    auto load = [&](int h, CtLoad<T>& L, FusedLoad<T>& X) {
        const long long c = base + (long long)wrap_idx(h, nd, g.bc) * sd;
        L.r0 = rho[c];
        L.m0 = md[c];
        L.bt = BT[c];
        L.rTm = rho[c + lo];
        L.mTm = md[c + lo];
        L.rTp = rho[c + hi];
        L.mTp = md[c + hi];
        L.bt1 = BT[c + hi];
        L.rXm = rho[c + xm_];
        L.mXm = md[c + xm_];
        L.rXp = rho[c + xp];
        L.mXp = md[c + xp];
        L.bx0 = BX[c];
        L.bx1 = BX[c + xp];
        X.bd = ld_own<NT>(&BD[base + (long long)wrap_idx(h - GB, nd, g.bc) * sd]);
        const long long cp = base + (long long)wrap_idx(h - GB - 1, nd, g.bc) * sd;
        X.me = ld_own<NT>(&mE[cp]);
        X.mf = ld_own<NT>(&mF[cp]);
        X.en = ld_own<NT>(&en[cp]);
    };

    EmfPipe<T> t0, t1, x0, x1;   // TA-face pencils (own, +TA), x-face pencils (own, +x)
    t0.clear();
    t1.clear();
    x0.clear();
    x1.clear();
    FluidPipe<T> P;
    P.clear();
    // rho and m_d of cells h-1 .. h-5 (the fluid head is h - 5)
    T rh[GB + 1], mh[GB + 1];
#pragma unroll
    for (int k = 0; k <= GB; k++) rh[k] = mh[k] = T(0);
    // new face fields of cell h - 5 (from the previous trip)
    T pD = T(0), pT0 = T(0), pT1 = T(0), pX0 = T(0), pX1 = T(0);
    CtLoad<T> cur;
    FusedLoad<T> curx;
    load(o0 - GCF, cur, curx);
    // unrolled 6 times, so that the shifts of the pipelines' register windows
    // become renames (FP64 0.66 -> 0.58 ms per launch at 256^3 against the
    // rolled loop; FP32 0.30 -> 0.26 ms)
#pragma unroll 6
    for (int h = o0 - GCF; h <= o1 + GCF; ++h) {
        CtLoad<T> nxt;
        FusedLoad<T> nxtx;
        load(h + 1, nxt, nxtx);
        // ---- field update (as in ct_march): EMFs at edge (h-4) + 1/2, new faces of cell q = h - 4
        const T r0 = cur.r0, m0 = cur.m0;
        const T rTm = cur.rTm, mTm = cur.mTm, rTp = cur.rTp, mTp = cur.mTp, bt1 = cur.bt1;
        const T bto = t0.B4, bxo = x0.B4, bt1o = t1.B4, bx1o = x1.B4;
        const T Gt0 = t0.push(qdiv(mTm + m0, rTm + r0), cur.bt, dt);
        const T Gt1 = t1.push(qdiv(m0 + mTp, r0 + rTp), bt1, dt);
        const T Gx0 = x0.push(qdiv(cur.mXm + m0, cur.rXm + r0), cur.bx0, dt);
        const T Gx1 = x1.push(qdiv(m0 + cur.mXp, r0 + cur.rXp), cur.bx1, dt);
        const T Ge0p = T_IS_E ? t0.G5 : x0.G5, Ge1p = T_IS_E ? t1.G5 : x1.G5;
        const T Gf0p = T_IS_E ? x0.G5 : t0.G5, Gf1p = T_IS_E ? x1.G5 : t1.G5;
        T nT0, nT1, nX0, nX1, nD;
        if (frozen) {
            nT0 = bto;
            nT1 = bt1o;
            nX0 = bxo;
            nX1 = bx1o;
            nD = curx.bd;
        } else {
            nT0 = bto - dt * (Gt0 - t0.G5);
            nT1 = bt1o - dt * (Gt1 - t1.G5);
            nX0 = bxo - dt * (Gx0 - x0.G5);
            nX1 = bx1o - dt * (Gx1 - x1.G5);
            nD = (curx.bd + dt * (Ge1p - Ge0p)) + dt * (Gf1p - Gf0p);
        }
        const int q = h - GB;
        if (active && q >= o0 && q < o1) {
            const long long cq = base + (long long)q * sd;
            put<NT>(&bout[E * N + cq], T_IS_E ? nT0 : nX0);
            put<NT>(&bout[F * N + cq], T_IS_E ? nX0 : nT0);
            put<NT>(&bout[D * N + cq], nD);
        }
        t0.G5 = Gt0;
        t1.G5 = Gt1;
        x0.G5 = Gx0;
        x1.G5 = Gx1;
        // ---- fluid update (as in fluid_march) of head p = h - 5 on the new field
        if (h >= o0 - GF + GB + 1) {
            const T bT = T(0.5) * (pT0 + pT1), bX = T(0.5) * (pX0 + pX1);
            T bh[3] = {T(0.5) * (pD + nD), T_IS_E ? bT : bX, T_IS_E ? bX : bT};
            const T uh[5] = {rh[GB], mh[GB], curx.me, curx.mf, curx.en};
            const T keep[5] = {P.u3[0], P.u3[1], P.u3[2], P.u3[3], P.u3[4]};
            const T bo[3] = {P.b3[0], P.b3[1], P.b3[2]};
            T un[5];
            P.push(uh, bh, gamma, dt, un);
            const int o = h - GB - 1 - GF;
            if (active && o >= o0) {
                if (frozen) {
#pragma unroll
                    for (int k = 0; k < 5; k++) un[k] = keep[k];
                }
                const long long co = base + (long long)o * sd;
                put<NT>(&uout[co], un[0]);
                put<NT>(&uout[(1 + D) * N + co], un[1]);
                put<NT>(&uout[(1 + E) * N + co], un[2]);
                put<NT>(&uout[(1 + F) * N + co], un[3]);
                put<NT>(&uout[4 * N + co], un[4]);
                if constexpr (CFL) {
                    const T cc = cfl_speed(un[0], un[1 + (3 - D) % 3], un[1 + (4 - D) % 3], un[1 + (5 - D) % 3],
                                           un[4], bo[(3 - D) % 3], bo[(4 - D) % 3], bo[(5 - D) % 3], gamma);
                    const unsigned long long bits = speed_bits(cc);
                    best = bits > best ? bits : best;
                }
            }
        }
        pD = nD;
        pT0 = nT0;
        pT1 = nT1;
        pX0 = nX0;
        pX1 = nX1;
#pragma unroll
        for (int k = GB; k > 0; k--) {
            rh[k] = rh[k - 1];
            mh[k] = mh[k - 1];
        }
        rh[0] = r0;
        mh[0] = m0;
        cur = nxt;
        curx = nxtx;
    }
    if constexpr (CFL) block_max_to_part<64 * MW>(best, threadIdx.x + 64 * threadIdx.y, part);
}

template <typename T, int D, bool CFL, bool NT>
__global__ void __launch_bounds__(64 * MW) ct_fluid_march(const T* __restrict__ uin, T* __restrict__ uout,
                                                          const T* __restrict__ bin, T* __restrict__ bout, Grid g,
                                                          T gamma, const Ctl* __restrict__ ctl, double dt_arg,
                                                          int chunk, unsigned long long* __restrict__ parts,
                                                          int* count)
{
    if constexpr (CFL) store_part_count(count);
    ct_fluid_march_body<T, D, CFL, NT>(uin, uout, bin, bout, g, gamma, ctl, dt_arg, chunk, blockIdx.x,
                                   parts + blockIdx.x);
}


// Neighbours along a row held in the lanes of one wavefront: lane i receives
// the value of lane i + 1 (lane_next) or lane i - 1 (lane_prev); what the end
// lane with no source receives is never used (a ghost lane of the wavefront
// form, or a lane the row form overwrites from LDS): with DPP it is 0 and
// otherwise its own value. DPP moves them with the whole-wavefront shifts
// (wave_shl:1 / wave_shr:1), one VALU move per 32 bits (writing 0 into the
// lane with no source, so the move needs no copy of its operand to keep that
// lane's old value); otherwise they go through the LDS crossbar
// (ds_bpermute), which costs no VALU issue slot but waits on LDS latency.
// Measured per kernel: DPP is 1.5-3 % faster for the FP64 fluid sweep and
// 10 % for the field part of the FP64 row-form fused sweep (0.538 -> 0.485 ms
// per launch at 256^3), the crossbar 20 % faster for the FP32 fluid sweep
// (closer to its issue limit); the FP32 field sweep shows no difference
// beyond run-to-run noise and keeps the crossbar.
__device__ __forceinline__ int dpp_next(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_prev(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xF, 0xF, true); }

template <bool DPP>
__device__ __forceinline__ float lane_next(float v)
{
    if constexpr (DPP) return __int_as_float(dpp_next(__float_as_int(v)));
    else return __shfl_down(v, 1);
}

template <bool DPP>
__device__ __forceinline__ float lane_prev(float v)
{
    if constexpr (DPP) return __int_as_float(dpp_prev(__float_as_int(v)));
    else return __shfl_up(v, 1);
}

template <bool DPP>
__device__ __forceinline__ double lane_next(double v)
{
    if constexpr (DPP) {
        const long long b = __double_as_longlong(v);
        const int lo = dpp_next((int)b), hi = dpp_next((int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    } else {
        return __shfl_down(v, 1);
    }
}

template <bool DPP>
__device__ __forceinline__ double lane_prev(double v)
{
    if constexpr (DPP) {
        const long long b = __double_as_longlong(v);
        const int lo = dpp_prev((int)b), hi = dpp_prev((int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    } else {
        return __shfl_up(v, 1);
    }
}

// ---------------------------------------------------------------------------
// fluid_x: a wavefront holds 64 consecutive cells of one row in its lanes (3
// ghost cells each side, so it updates XW = 58 of them) and takes every
// stencil neighbour from the adjacent lane with a cross-lane shuffle; the
// wavefronts are independent (no LDS, no barrier until the final c_max
// reduction). Workgroups of 4 wavefronts; logical workgroup lb covers
// wavefronts 4 lb .. 4 lb + 3, rows fastest in segments along x. (Staging
// rows in LDS with a barrier per stage measured 24 % slower.)
constexpr int XW = 64 - 2 * GF;

template <typename T, bool CFL, bool NT = true>
__device__ __forceinline__ void fluid_x_body(const T* __restrict__ uin, T* __restrict__ uout,
                                             const T* __restrict__ bf, const Grid& g, T gamma,
                                             const Ctl* __restrict__ ctl, double dt_arg, unsigned lb,
                                             unsigned long long* __restrict__ part)
{
    const int lane = threadIdx.x & 63;
    const int nx = g.n[0], ny = g.n[1];
    // wavefront-uniform indices (scalar registers); 32 bits suffice, since a
    // grid that fits in device memory has fewer than 2^32 wavefronts
    const unsigned wpr = (unsigned)(nx + XW - 1) / XW;   // wavefronts per row
    const unsigned nrows = (unsigned)ny * (unsigned)g.n[2];
    const unsigned wave = lb * 4u + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned row = wave / wpr;
    const int seg = (int)(wave - row * wpr);
    const bool live = row < nrows;        // wavefronts past the last row only join the block reduction
    const unsigned rowc = live ? row : 0u;
    const int j = (int)(rowc % (unsigned)ny), k = (int)(rowc / (unsigned)ny);
    const int xu = seg * XW - GF + lane;  // position along x before the boundary map
    const int x = wrap_idx(xu, nx, g.bc), xn = wrap_idx(xu + 1, nx, g.bc);
    const long long N = g.N;
    const long long rb = (long long)nx * (j + (long long)ny * k);
    const long long c = rb + x;
    const long long cy = (long long)nx * (wrap_idx(j + 1, ny, g.bc) + (long long)ny * k) + x;
    const long long cz = (long long)nx * (j + (long long)ny * wrap_idx(k + 1, g.n[2], g.bc)) + x;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;
    constexpr bool kDpp = kExact<T>;

    T u[5], b[3], rr[5], ll[5];
#pragma unroll
    for (int q = 0; q < 5; q++) u[q] = uin[q * N + c];
    b[0] = T(0.5) * (bf[c] + bf[rb + xn]);
    b[1] = T(0.5) * (bf[N + c] + bf[N + cy]);
    b[2] = T(0.5) * (bf[2 * N + c] + bf[2 * N + cz]);
    movers(u, b, gamma, rr, ll);
    // stage 1: first-order flux at x + 1/2, half step, movers of the half state
    T f[5], uh[5], rp[5], lp[5];
#pragma unroll
    for (int q = 0; q < 5; q++) f[q] = rr[q] - lane_next<kDpp>(ll[q]);
#pragma unroll
    for (int q = 0; q < 5; q++) uh[q] = u[q] - (dt * T(0.5)) * (f[q] - lane_prev<kDpp>(f[q]));
    movers(uh, b, gamma, rp, lp);
    // stage 2: limited movers (eq. limiter on half-differences)
    T Rr[5], Ll[5];
#pragma unroll
    for (int q = 0; q < 5; q++) {
        const T a = lane_prev<kDpp>(rp[q]), c0 = rp[q], d = lane_next<kDpp>(rp[q]);
        Rr[q] = c0 + vanleer_half(c0 - a, d - c0);
        const T al = lane_prev<kDpp>(lp[q]), cl = lp[q], dl = lane_next<kDpp>(lp[q]);
        Ll[q] = cl - vanleer_half(cl - al, dl - cl);
    }
    // full update of lanes GF .. GF + XW - 1 (eq. Delta_u_full)
    T fp[5], un[5];
#pragma unroll
    for (int q = 0; q < 5; q++) fp[q] = Rr[q] - lane_next<kDpp>(Ll[q]);
#pragma unroll
    for (int q = 0; q < 5; q++) {
        const T fm = lane_prev<kDpp>(fp[q]);
        un[q] = frozen ? u[q] : u[q] - dt * (fp[q] - fm);
    }
    unsigned long long best = 0ull;
    if (live && lane >= GF && lane < GF + XW && xu < nx) {
#pragma unroll
        for (int q = 0; q < 5; q++) put<NT>(&uout[q * N + c], un[q]);
        if constexpr (CFL) {
            const T cc = cfl_speed(un[0], un[1], un[2], un[3], un[4], b[0], b[1], b[2], gamma);
            best = speed_bits(cc);
        }
    }
    if constexpr (CFL) block_max_to_part<256>(best, threadIdx.x, part);
}

template <typename T, bool CFL, bool NT>
__global__ void __launch_bounds__(256) fluid_x_wave(const T* __restrict__ uin, T* __restrict__ uout,
                                                    const T* __restrict__ bf, Grid g, T gamma,
                                                    const Ctl* __restrict__ ctl, double dt_arg,
                                                    unsigned long long* __restrict__ parts, int* count)
{
    if constexpr (CFL) store_part_count(count);
    fluid_x_body<T, CFL, NT>(uin, uout, bf, g, gamma, ctl, dt_arg, blockIdx.x, parts + blockIdx.x);
}

static unsigned x_wave_blocks(const Grid& g)
{
    const long long waves = (long long)g.n[1] * g.n[2] * ((g.n[0] + XW - 1) / XW);
    return (unsigned)((waves + 3) / 4);
}

// B_{y->x}, B_{z->x}: a wavefront holds 64 consecutive cells of one row (4
// ghost cells each side, so it updates XWC = 56) and runs the four EMF
// pencils of the row (own and +y face for B_y, own and +z face for B_z) stage
// by stage, with cross-lane shuffles for the neighbours along x.
constexpr int XWC = 64 - 2 * GB;

template <typename T, bool NT = true>
__device__ __forceinline__ void ct_x_body(const T* __restrict__ uf, const T* __restrict__ bin,
                                          T* __restrict__ bout, const Grid& g, const Ctl* __restrict__ ctl,
                                          double dt_arg, unsigned lb)
{
    const int lane = threadIdx.x & 63;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const unsigned wpr = (unsigned)(nx + XWC - 1) / XWC;
    const unsigned nrows = (unsigned)ny * (unsigned)nz;
    const unsigned wave = lb * 4u + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned row = wave / wpr;
    if (row >= nrows) return;   // no barrier follows: whole wavefronts past the last row leave
    const int seg = (int)(wave - row * wpr);
    const int j = (int)(row % (unsigned)ny), k = (int)(row / (unsigned)ny);
    const int xu = seg * XWC - GB + lane;
    const int x = wrap_idx(xu, nx, g.bc);
    const int jm = wrap_idx(j - 1, ny, g.bc), jp = wrap_idx(j + 1, ny, g.bc);
    const int km = wrap_idx(k - 1, nz, g.bc), kp = wrap_idx(k + 1, nz, g.bc);
    const long long N = g.N;
    const long long c = (long long)nx * (j + (long long)ny * k) + x;
    const long long cym = (long long)nx * (jm + (long long)ny * k) + x;
    const long long cyp = (long long)nx * (jp + (long long)ny * k) + x;
    const long long czm = (long long)nx * (j + (long long)ny * km) + x;
    const long long czp = (long long)nx * (j + (long long)ny * kp) + x;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;

    // pencil e: 0 = B_y own, 1 = B_y at +y, 2 = B_z own, 3 = B_z at +z
    T vh[4], Bk[4];
    const T r0 = uf[c], m0 = uf[N + c];
    vh[0] = qdiv(uf[N + cym] + m0, uf[cym] + r0);
    vh[1] = qdiv(m0 + uf[N + cyp], r0 + uf[cyp]);
    vh[2] = qdiv(uf[N + czm] + m0, uf[czm] + r0);
    vh[3] = qdiv(m0 + uf[N + czp], r0 + uf[czp]);
    Bk[0] = bin[N + c];
    Bk[1] = bin[N + cyp];
    Bk[2] = bin[2 * N + c];
    Bk[3] = bin[2 * N + czp];
    T G[4], gm[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        // smoothed velocity (eq. averaging_x) and v B
        const T vv = T(0.25) * (lane_prev<false>(vh[e]) + T(2) * vh[e] + lane_next<false>(vh[e]));
        const T qb = vv * Bk[e];
        // edge velocity and first-order upwind EMF at x + 1/2
        const T ev = T(0.5) * (vv + lane_next<false>(vv));
        const T qbn = lane_next<false>(qb);
        const T g1 = ev > T(0) ? qb : qbn;
        // half step and v B^{t+dt/2}
        const T bhalf = Bk[e] - (dt * T(0.5)) * (g1 - lane_prev<false>(g1));
        const T qh = vv * bhalf;
        // limited slope and second-order EMF at x + 1/2
        const T qhm = lane_prev<false>(qh), qhp = lane_next<false>(qh);
        const T sq = vanleer_half(qh - qhm, qhp - qh);
        const T sqp = lane_next<false>(sq);
        G[e] = ev > T(0) ? qh + sq : qhp - sqp;
        gm[e] = lane_prev<false>(G[e]);
    }
    // advection of B_y, B_z and constraint update of B_x
    if (lane >= GB && lane < GB + XWC && xu < nx) {
        const T bx = bin[c];
        // a frozen state (status set) is copied through unchanged
        const T ny0 = frozen ? Bk[0] : Bk[0] - dt * (G[0] - gm[0]);
        const T nz0 = frozen ? Bk[2] : Bk[2] - dt * (G[2] - gm[2]);
        const T nx0 = frozen ? bx : (bx + dt * (gm[1] - gm[0])) + dt * (gm[3] - gm[2]);
        put<NT>(&bout[N + c], ny0);
        put<NT>(&bout[2 * N + c], nz0);
        put<NT>(&bout[c], nx0);
    }
}

template <typename T, bool NT>
__global__ void __launch_bounds__(256) ct_x_wave(const T* __restrict__ uf, const T* __restrict__ bin,
                                                 T* __restrict__ bout, Grid g, const Ctl* __restrict__ ctl,
                                                 double dt_arg)
{
    ct_x_body<T, NT>(uf, bin, bout, g, ctl, dt_arg, blockIdx.x);
}

static unsigned ct_x_wave_blocks(const Grid& g)
{
    const long long waves = (long long)g.n[1] * g.n[2] * ((g.n[0] + XWC - 1) / XWC);
    return (unsigned)((waves + 3) / 4);
}

// Reverse L_x on periodic grids (Sec. 4.3: field update, then fluid update)
// in one wavefront pass: the field update of ct_x_body on 64 consecutive
// cells of a row, then the fluid update of fluid_x_body on the new field held
// in the lanes. The new faces are valid on lanes 4 .. 59; the fluid update of
// lane L reads the centred field on lanes L - 3 .. L + 3 (B_x up to L + 4), so
// lanes 7 .. 55 are stored: XWF = 49 cells per wavefront. Same expressions as
// the two separate kernels, so the same bits; periodic wrapping makes the new
// field of a ghost lane that of the cell it maps to.
constexpr int XWF = 64 - 2 * GCF - 1;

template <typename T, bool CFL, bool NT = true>
__device__ __forceinline__ void ct_fluid_x_body(const T* __restrict__ uin, T* __restrict__ uout,
                                                const T* __restrict__ bin, T* __restrict__ bout, const Grid& g,
                                                T gamma, const Ctl* __restrict__ ctl, double dt_arg, unsigned lb,
                                                unsigned long long* __restrict__ part)
{
    const int lane = threadIdx.x & 63;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const unsigned wpr = (unsigned)(nx + XWF - 1) / XWF;
    const unsigned nrows = (unsigned)ny * (unsigned)nz;
    const unsigned wave = lb * 4u + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned row = wave / wpr;
    const int seg = (int)(wave - row * wpr);
    const bool live = row < nrows;        // wavefronts past the last row only join the block reduction
    const unsigned rowc = live ? row : 0u;
    const int j = (int)(rowc % (unsigned)ny), k = (int)(rowc / (unsigned)ny);
    const int xu = seg * XWF - GCF + lane;
    const int x = wrap_idx(xu, nx, g.bc);
    const int jm = wrap_idx(j - 1, ny, g.bc), jp = wrap_idx(j + 1, ny, g.bc);
    const int km = wrap_idx(k - 1, nz, g.bc), kp = wrap_idx(k + 1, nz, g.bc);
    const long long N = g.N;
    const long long c = (long long)nx * (j + (long long)ny * k) + x;
    const long long cym = (long long)nx * (jm + (long long)ny * k) + x;
    const long long cyp = (long long)nx * (jp + (long long)ny * k) + x;
    const long long czm = (long long)nx * (j + (long long)ny * km) + x;
    const long long czp = (long long)nx * (j + (long long)ny * kp) + x;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;
    constexpr bool kDpp = kExact<T>;

    // ---- field update (as in ct_x_body)
    T vh[4], Bk[4];
    const T r0 = uin[c], m0 = uin[N + c];
    vh[0] = qdiv(uin[N + cym] + m0, uin[cym] + r0);
    vh[1] = qdiv(m0 + uin[N + cyp], r0 + uin[cyp]);
    vh[2] = qdiv(uin[N + czm] + m0, uin[czm] + r0);
    vh[3] = qdiv(m0 + uin[N + czp], r0 + uin[czp]);
    Bk[0] = bin[N + c];
    Bk[1] = bin[N + cyp];
    Bk[2] = bin[2 * N + c];
    Bk[3] = bin[2 * N + czp];
    const T bx = bin[c];
    T u[5];
    u[0] = r0;
    u[1] = m0;
    u[2] = uin[2 * N + c];
    u[3] = uin[3 * N + c];
    u[4] = uin[4 * N + c];
    T G[4], gm[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const T vv = T(0.25) * (lane_prev<false>(vh[e]) + T(2) * vh[e] + lane_next<false>(vh[e]));
        const T qb = vv * Bk[e];
        const T ev = T(0.5) * (vv + lane_next<false>(vv));
        const T qbn = lane_next<false>(qb);
        const T g1 = ev > T(0) ? qb : qbn;
        const T bhalf = Bk[e] - (dt * T(0.5)) * (g1 - lane_prev<false>(g1));
        const T qh = vv * bhalf;
        const T qhm = lane_prev<false>(qh), qhp = lane_next<false>(qh);
        const T sq = vanleer_half(qh - qhm, qhp - qh);
        const T sqp = lane_next<false>(sq);
        G[e] = ev > T(0) ? qh + sq : qhp - sqp;
        gm[e] = lane_prev<false>(G[e]);
    }
    // new faces: B_y, B_z of this row and of the +y / +z rows, B_x
    T nB[5];   // B_x, B_y, B_y(+y), B_z, B_z(+z)
    if (frozen) {
        nB[0] = bx;
        nB[1] = Bk[0];
        nB[2] = Bk[1];
        nB[3] = Bk[2];
        nB[4] = Bk[3];
    } else {
        nB[1] = Bk[0] - dt * (G[0] - gm[0]);
        nB[2] = Bk[1] - dt * (G[1] - gm[1]);
        nB[3] = Bk[2] - dt * (G[2] - gm[2]);
        nB[4] = Bk[3] - dt * (G[3] - gm[3]);
        nB[0] = (bx + dt * (gm[1] - gm[0])) + dt * (gm[3] - gm[2]);
    }
    const bool store = live && lane >= GCF && lane < GCF + XWF && xu < nx;
    if (store) {
        put<NT>(&bout[c], nB[0]);
        put<NT>(&bout[N + c], nB[1]);
        put<NT>(&bout[2 * N + c], nB[3]);
    }
    // ---- fluid update (as in fluid_x_body) on the new field
    T b[3], rr[5], ll[5];
    b[0] = T(0.5) * (nB[0] + lane_next<kDpp>(nB[0]));
    b[1] = T(0.5) * (nB[1] + nB[2]);
    b[2] = T(0.5) * (nB[3] + nB[4]);
    movers(u, b, gamma, rr, ll);
    T f[5], uh[5], rp[5], lp[5];
#pragma unroll
    for (int q = 0; q < 5; q++) f[q] = rr[q] - lane_next<kDpp>(ll[q]);
#pragma unroll
    for (int q = 0; q < 5; q++) uh[q] = u[q] - (dt * T(0.5)) * (f[q] - lane_prev<kDpp>(f[q]));
    movers(uh, b, gamma, rp, lp);
    T Rr[5], Ll[5];
#pragma unroll
    for (int q = 0; q < 5; q++) {
        const T a = lane_prev<kDpp>(rp[q]), c0 = rp[q], d = lane_next<kDpp>(rp[q]);
        Rr[q] = c0 + vanleer_half(c0 - a, d - c0);
        const T al = lane_prev<kDpp>(lp[q]), cl = lp[q], dl = lane_next<kDpp>(lp[q]);
        Ll[q] = cl - vanleer_half(cl - al, dl - cl);
    }
    T fp[5], un[5];
#pragma unroll
    for (int q = 0; q < 5; q++) fp[q] = Rr[q] - lane_next<kDpp>(Ll[q]);
#pragma unroll
    for (int q = 0; q < 5; q++) {
        const T fm = lane_prev<kDpp>(fp[q]);
        un[q] = frozen ? u[q] : u[q] - dt * (fp[q] - fm);
    }
    unsigned long long best = 0ull;
    if (store) {
#pragma unroll
        for (int q = 0; q < 5; q++) put<NT>(&uout[q * N + c], un[q]);
        if constexpr (CFL) {
            const T cc = cfl_speed(un[0], un[1], un[2], un[3], un[4], b[0], b[1], b[2], gamma);
            best = speed_bits(cc);
        }
    }
    if constexpr (CFL) block_max_to_part<256>(best, threadIdx.x, part);
}

template <typename T, bool CFL, bool NT>
__global__ void __launch_bounds__(256) ct_fluid_x_wave(const T* __restrict__ uin, T* __restrict__ uout,
                                                       const T* __restrict__ bin, T* __restrict__ bout, Grid g,
                                                       T gamma, const Ctl* __restrict__ ctl, double dt_arg,
                                                       unsigned long long* __restrict__ parts, int* count)
{
    if constexpr (CFL) store_part_count(count);
    ct_fluid_x_body<T, CFL, NT>(uin, uout, bin, bout, g, gamma, ctl, dt_arg, blockIdx.x, parts + blockIdx.x);
}

static unsigned ct_fluid_x_blocks(const Grid& g)
{
    const long long waves = (long long)g.n[1] * g.n[2] * ((g.n[0] + XWF - 1) / XWF);
    return (unsigned)((waves + 3) / 4);
}

// ---------------------------------------------------------------------------
// Reverse L_x on periodic rows whose length is a multiple of 64 (up to
// 64 * XRW): one workgroup holds a whole row, one cell per lane, with no halo
// lanes. Neighbours along x come from the adjacent lane inside a wavefront;
// the two end lanes of a wavefront take theirs from the neighbouring
// wavefronts (cyclically: the row is periodic) through LDS, one barrier per
// exchange (two buffers alternate, so one barrier orders each exchange).
// Every value is computed by the same expressions as in ct_fluid_x_body, so
// the result is the same bit for bit; the halo lanes of the wavefront form
// (15 of 64, and a sixth wavefront per 256-cell row) are gone, which is what
// limits that form (it is bound by instruction issue).
constexpr int XRW = 8;     // wavefronts per row workgroup at most (rows up to 512 cells)
constexpr int XRV = 10;    // values per exchange at most

template <typename T>
struct RowX {
    T (*xb)[2][XRW][XRV];  // [buffer][0: first lane, 1: last lane][wavefront][value]
    int buf, w, W, lane;

    // nxt[k] = v[k] of cell i + 1 and / or prv[k] = v[k] of cell i - 1
    template <int K, bool NEXT, bool PREV, bool DPP>
    __device__ __forceinline__ void shift(const T* v, T* nxt, T* prv)
    {
#pragma unroll
        for (int k = 0; k < K; k++) {
            if constexpr (NEXT) nxt[k] = lane_next<DPP>(v[k]);
            if constexpr (PREV) prv[k] = lane_prev<DPP>(v[k]);
        }
        if (NEXT && lane == 0) {
#pragma unroll
            for (int k = 0; k < K; k++) xb[buf][0][w][k] = v[k];
        }
        if (PREV && lane == 63) {
#pragma unroll
            for (int k = 0; k < K; k++) xb[buf][1][w][k] = v[k];
        }
        __syncthreads();
        if (NEXT && lane == 63) {
            const int wn = w + 1 == W ? 0 : w + 1;
#pragma unroll
            for (int k = 0; k < K; k++) nxt[k] = xb[buf][0][wn][k];
        }
        if (PREV && lane == 0) {
            const int wp = w == 0 ? W - 1 : w - 1;
#pragma unroll
            for (int k = 0; k < K; k++) prv[k] = xb[buf][1][wp][k];
        }
        buf ^= 1;
    }
};

template <typename T, bool CFL, bool NT>
__global__ void __launch_bounds__(64 * XRW) ct_fluid_x_row(const T* __restrict__ uin, T* __restrict__ uout,
                                                           const T* __restrict__ bin, T* __restrict__ bout, Grid g,
                                                           T gamma, const Ctl* __restrict__ ctl, double dt_arg,
                                                           unsigned long long* __restrict__ parts, int* count)
{
    __shared__ T xb[2][2][XRW][XRV];
    __shared__ unsigned long long wmax[XRW];
    if constexpr (CFL) store_part_count(count);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const unsigned row = blockIdx.x;
    const int j = (int)(row % (unsigned)ny), k = (int)(row / (unsigned)ny);
    const int x = 64 * w + lane;
    const int jm = wrap_idx(j - 1, ny, g.bc), jp = wrap_idx(j + 1, ny, g.bc);
    const int km = wrap_idx(k - 1, nz, g.bc), kp = wrap_idx(k + 1, nz, g.bc);
    const long long N = g.N;
    const long long c = (long long)nx * (j + (long long)ny * k) + x;
    const long long cym = (long long)nx * (jm + (long long)ny * k) + x;
    const long long cyp = (long long)nx * (jp + (long long)ny * k) + x;
    const long long czm = (long long)nx * (j + (long long)ny * km) + x;
    const long long czp = (long long)nx * (j + (long long)ny * kp) + x;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;
    constexpr bool kDpp = kExact<T>;
    RowX<T> X{xb, 0, w, W, lane};

    // ---- field update (as in ct_x_body)
    T vh[4], Bk[4];
    const T r0 = uin[c], m0 = uin[N + c];
    vh[0] = qdiv(uin[N + cym] + m0, uin[cym] + r0);
    vh[1] = qdiv(m0 + uin[N + cyp], r0 + uin[cyp]);
    vh[2] = qdiv(uin[N + czm] + m0, uin[czm] + r0);
    vh[3] = qdiv(m0 + uin[N + czp], r0 + uin[czp]);
    Bk[0] = bin[N + c];
    Bk[1] = bin[N + cyp];
    Bk[2] = bin[2 * N + c];
    Bk[3] = bin[2 * N + czp];
    const T bx = ld_own<NT>(&bin[c]);
    T u[5];
    u[0] = r0;
    u[1] = m0;
    u[2] = ld_own<NT>(&uin[2 * N + c]);
    u[3] = ld_own<NT>(&uin[3 * N + c]);
    u[4] = ld_own<NT>(&uin[4 * N + c]);
    T vhn[4], vhp[4];
    X.template shift<4, true, true, kDpp>(vh, vhn, vhp);
    T vv[4], qb[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        vv[e] = T(0.25) * (vhp[e] + T(2) * vh[e] + vhn[e]);
        qb[e] = vv[e] * Bk[e];
    }
    T t8[8], t8n[8];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        t8[e] = vv[e];
        t8[4 + e] = qb[e];
    }
    X.template shift<8, true, false, kDpp>(t8, t8n, nullptr);
    T ev[4], g1[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        ev[e] = T(0.5) * (vv[e] + t8n[e]);
        g1[e] = ev[e] > T(0) ? qb[e] : t8n[4 + e];
    }
    T g1p[4];
    X.template shift<4, false, true, kDpp>(g1, nullptr, g1p);
    T qh[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const T bhalf = Bk[e] - (dt * T(0.5)) * (g1[e] - g1p[e]);
        qh[e] = vv[e] * bhalf;
    }
    T qhn[4], qhp[4];
    X.template shift<4, true, true, kDpp>(qh, qhn, qhp);
    T sq[4];
#pragma unroll
    for (int e = 0; e < 4; e++) sq[e] = vanleer_half(qh[e] - qhp[e], qhn[e] - qh[e]);
    T sqn[4];
    X.template shift<4, true, false, kDpp>(sq, sqn, nullptr);
    T G[4];
#pragma unroll
    for (int e = 0; e < 4; e++) G[e] = ev[e] > T(0) ? qh[e] + sq[e] : qhn[e] - sqn[e];
    T gm[4];
    X.template shift<4, false, true, kDpp>(G, nullptr, gm);
    T nB[5];   // B_x, B_y, B_y(+y), B_z, B_z(+z)
    if (frozen) {
        nB[0] = bx;
        nB[1] = Bk[0];
        nB[2] = Bk[1];
        nB[3] = Bk[2];
        nB[4] = Bk[3];
    } else {
        nB[1] = Bk[0] - dt * (G[0] - gm[0]);
        nB[2] = Bk[1] - dt * (G[1] - gm[1]);
        nB[3] = Bk[2] - dt * (G[2] - gm[2]);
        nB[4] = Bk[3] - dt * (G[3] - gm[3]);
        nB[0] = (bx + dt * (gm[1] - gm[0])) + dt * (gm[3] - gm[2]);
    }
    put<NT>(&bout[c], nB[0]);
    put<NT>(&bout[N + c], nB[1]);
    put<NT>(&bout[2 * N + c], nB[3]);
    // ---- fluid update (as in fluid_x_body) on the new field
    T bxn;
    X.template shift<1, true, false, kDpp>(nB, &bxn, nullptr);
    T b[3], rr[5], ll[5];
    b[0] = T(0.5) * (nB[0] + bxn);
    b[1] = T(0.5) * (nB[1] + nB[2]);
    b[2] = T(0.5) * (nB[3] + nB[4]);
    movers(u, b, gamma, rr, ll);
    T lln[5];
    X.template shift<5, true, false, kDpp>(ll, lln, nullptr);
    T f[5];
#pragma unroll
    for (int q = 0; q < 5; q++) f[q] = rr[q] - lln[q];
    T fpv[5];
    X.template shift<5, false, true, kDpp>(f, nullptr, fpv);
    T uh[5], rp[5], lp[5];
#pragma unroll
    for (int q = 0; q < 5; q++) uh[q] = u[q] - (dt * T(0.5)) * (f[q] - fpv[q]);
    movers(uh, b, gamma, rp, lp);
    T t10[10], t10n[10], t10p[10];
#pragma unroll
    for (int q = 0; q < 5; q++) {
        t10[q] = rp[q];
        t10[5 + q] = lp[q];
    }
    X.template shift<10, true, true, kDpp>(t10, t10n, t10p);
    T Rr[5], Ll[5];
#pragma unroll
    for (int q = 0; q < 5; q++) {
        const T a = t10p[q], c0 = rp[q], d = t10n[q];
        Rr[q] = c0 + vanleer_half(c0 - a, d - c0);
        const T al = t10p[5 + q], cl = lp[q], dl = t10n[5 + q];
        Ll[q] = cl - vanleer_half(cl - al, dl - cl);
    }
    T Lln[5];
    X.template shift<5, true, false, kDpp>(Ll, Lln, nullptr);
    T fp[5];
#pragma unroll
    for (int q = 0; q < 5; q++) fp[q] = Rr[q] - Lln[q];
    T fm[5];
    X.template shift<5, false, true, kDpp>(fp, nullptr, fm);
    T un[5];
#pragma unroll
    for (int q = 0; q < 5; q++) un[q] = frozen ? u[q] : u[q] - dt * (fp[q] - fm[q]);
#pragma unroll
    for (int q = 0; q < 5; q++) put<NT>(&uout[q * N + c], un[q]);
    if constexpr (CFL) {
        const T cc = cfl_speed(un[0], un[1], un[2], un[3], un[4], b[0], b[1], b[2], gamma);
        unsigned long long best = wave_max_u64(speed_bits(cc));
        if (lane == 0) wmax[w] = best;
        __syncthreads();
        if (threadIdx.x < 64) {
            best = (int)threadIdx.x < W ? wmax[threadIdx.x] : 0ull;
            best = wave_max_u64(best);
            if (threadIdx.x == 0) parts[blockIdx.x] = best;
        }
    }
}

// The row form applies to periodic rows of 64 k cells, k <= XRW, in FP64,
// where the wavefront form is bound by instruction issue: 0.607 -> 0.545 ms
// per launch at 256^3. In FP32 the twelve barriers cost more than the halo
// lanes save (0.348 -> 0.372 ms); FP32 runs the lane-row form instead.
template <typename T>
static bool ct_fluid_x_row_ok(const Grid& g)
{
    return kExact<T> && g.bc == 0 && g.n[0] % 64 == 0 && g.n[0] <= 64 * XRW;
}

// fluid_x alone in the row form (FP64 periodic rows of 64 k cells, k <= XRW):
// one workgroup per row, one cell per lane, neighbours across the
// wavefront ends exchanged through LDS (six exchanges); the same expressions
// as fluid_x_body, so the same bits. The wavefront form spends 320 lanes on
// a 256-cell row (5 wavefronts of 58 stored cells).
template <typename T, bool CFL, bool NT>
__global__ void __launch_bounds__(64 * XRW) fluid_x_row(const T* __restrict__ uin, T* __restrict__ uout,
                                                        const T* __restrict__ bf, Grid g, T gamma,
                                                        const Ctl* __restrict__ ctl, double dt_arg,
                                                        unsigned long long* __restrict__ parts, int* count)
{
    __shared__ T xb[2][2][XRW][XRV];
    __shared__ unsigned long long wmax[XRW];
    if constexpr (CFL) store_part_count(count);
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int W = blockDim.x >> 6;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const unsigned row = blockIdx.x;
    const int j = (int)(row % (unsigned)ny), k = (int)(row / (unsigned)ny);
    const int x = 64 * w + lane;
    const int jp = wrap_idx(j + 1, ny, g.bc), kp = wrap_idx(k + 1, nz, g.bc);
    const long long N = g.N;
    const long long c = (long long)nx * (j + (long long)ny * k) + x;
    const long long cyp = (long long)nx * (jp + (long long)ny * k) + x;
    const long long czp = (long long)nx * (j + (long long)ny * kp) + x;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;
    constexpr bool kDpp = kExact<T>;
    RowX<T> X{xb, 0, w, W, lane};

    T u[5];
#pragma unroll
    for (int q = 0; q < 5; q++) u[q] = ld_own<NT>(&uin[q * N + c]);
    const T bx = ld_own<NT>(&bf[c]);
    T b[3];
    b[1] = T(0.5) * (bf[N + c] + bf[N + cyp]);
    b[2] = T(0.5) * (bf[2 * N + c] + bf[2 * N + czp]);
    T bxn;
    X.template shift<1, true, false, kDpp>(&bx, &bxn, nullptr);
    b[0] = T(0.5) * (bx + bxn);
    T rr[5], ll[5];
    movers(u, b, gamma, rr, ll);
    T lln[5];
    X.template shift<5, true, false, kDpp>(ll, lln, nullptr);
    T f[5];
#pragma unroll
    for (int q = 0; q < 5; q++) f[q] = rr[q] - lln[q];
    T fpv[5];
    X.template shift<5, false, true, kDpp>(f, nullptr, fpv);
    T uh[5], rp[5], lp[5];
#pragma unroll
    for (int q = 0; q < 5; q++) uh[q] = u[q] - (dt * T(0.5)) * (f[q] - fpv[q]);
    movers(uh, b, gamma, rp, lp);
    T t10[10], t10n[10], t10p[10];
#pragma unroll
    for (int q = 0; q < 5; q++) {
        t10[q] = rp[q];
        t10[5 + q] = lp[q];
    }
    X.template shift<10, true, true, kDpp>(t10, t10n, t10p);
    T Rr[5], Ll[5];
#pragma unroll
    for (int q = 0; q < 5; q++) {
        const T a = t10p[q], c0 = rp[q], d = t10n[q];
        Rr[q] = c0 + vanleer_half(c0 - a, d - c0);
        const T al = t10p[5 + q], cl = lp[q], dl = t10n[5 + q];
        Ll[q] = cl - vanleer_half(cl - al, dl - cl);
    }
    T Lln[5];
    X.template shift<5, true, false, kDpp>(Ll, Lln, nullptr);
    T fp[5];
#pragma unroll
    for (int q = 0; q < 5; q++) fp[q] = Rr[q] - Lln[q];
    T fm[5];
    X.template shift<5, false, true, kDpp>(fp, nullptr, fm);
    T un[5];
#pragma unroll
    for (int q = 0; q < 5; q++) un[q] = frozen ? u[q] : u[q] - dt * (fp[q] - fm[q]);
#pragma unroll
    for (int q = 0; q < 5; q++) put<NT>(&uout[q * N + c], un[q]);
    if constexpr (CFL) {
        const T cc = cfl_speed(un[0], un[1], un[2], un[3], un[4], b[0], b[1], b[2], gamma);
        unsigned long long best = wave_max_u64(speed_bits(cc));
        if (lane == 0) wmax[w] = best;
        __syncthreads();
        if (threadIdx.x < 64) {
            best = (int)threadIdx.x < W ? wmax[threadIdx.x] : 0ull;
            best = wave_max_u64(best);
            if (threadIdx.x == 0) parts[blockIdx.x] = best;
        }
    }
}

// ---------------------------------------------------------------------------
// x sweeps on periodic rows of 64 K cells in FP32, lane-row form: one
// wavefront holds a whole row, K cells per lane (cell x = lane + 64 s in set
// s), so no lane is a halo lane and nothing crosses wavefronts. The x
// neighbour of a cell is the same set's value one lane over, rotated within
// the wavefront, except at the seam lane (63 for the next cell, 0 for the
// previous one), which takes the adjacent set's rotated value (cyclically).
// Used for the fused reverse L_x (ct_fluid_x_lrow: 0.350 -> 0.255 ms per
// launch at 256^3), the field update along x (ct_x_lrow: 0.169 -> 0.120 ms)
// and the fluid update along x (fluid_x_lrow: 0.187 -> 0.157 ms, against the
// wavefront form whose 6 halo lanes of 64 update nothing). Same expressions
// as the wavefront forms, so the same bits.
// The seam selects take their set indices as template constants (an index
// sequence, not a loop): with a loop index the compiler folds the select of
// two set values, r[a] or r[b], into a select of the index followed by an
// indexed pick among all K values, K - 1 selects more per value.
template <typename T, int K, int SH, int... Q>
__device__ __forceinline__ void lrow_seam(const T* r, T* out, bool seam, std::integer_sequence<int, Q...>)
{
    ((out[Q] = seam ? r[(Q + SH) % K] : r[Q]), ...);
}

// Lanes of a lane-row wavefront: 64 / W rows of W lanes each (W = 16, 32 or
// 64), K cells per lane; cell x of set s is xl + W s.
template <int W>
struct LRowLanes {
    int xl;                      // position of the lane among its row's lanes
    int src_next, src_prev;      // lanes holding the next / previous cell of the same set
    bool seam_next, seam_prev;   // the neighbour is in the adjacent set instead
};

template <int W>
__device__ __forceinline__ LRowLanes<W> lrow_lanes()
{
    LRowLanes<W> L;
    const int lane = threadIdx.x & 63;
    const int first = lane & ~(W - 1);
    L.xl = lane & (W - 1);
    L.src_next = first | ((lane + 1) & (W - 1));
    L.src_prev = first | ((lane + W - 1) & (W - 1));
    L.seam_next = L.xl == W - 1;
    L.seam_prev = L.xl == 0;
    return L;
}

template <int W>
__device__ __forceinline__ int lrow_x(const LRowLanes<W>& L, int q) { return L.xl + W * q; }

// With one row per wavefront (W = 64) the source lanes are a rotation of the
// wavefront by one lane, which the FP64 sweeps take with the DPP whole-
// wavefront rotates (wave_rol:1 / wave_ror:1) instead of the LDS crossbar.
template <typename T>
constexpr bool kLRowDpp = kExact<T>;

__device__ __forceinline__ int dpp_rol(int v) { return __builtin_amdgcn_mov_dpp(v, 0x134, 0xF, 0xF, false); }
__device__ __forceinline__ int dpp_ror(int v) { return __builtin_amdgcn_mov_dpp(v, 0x13C, 0xF, 0xF, false); }

template <bool NEXT>
__device__ __forceinline__ float lane_rot(float v)
{
    return __int_as_float(NEXT ? dpp_rol(__float_as_int(v)) : dpp_ror(__float_as_int(v)));
}

template <bool NEXT>
__device__ __forceinline__ double lane_rot(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = NEXT ? dpp_rol((int)b) : dpp_ror((int)b);
    const int hi = NEXT ? dpp_rol((int)(b >> 32)) : dpp_ror((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <typename T, int K, int W>
__device__ __forceinline__ void lrow_next(const T* v, T* out, const LRowLanes<W>& L)
{
    T r[K];
#pragma unroll
    for (int q = 0; q < K; q++) {
        if constexpr (W == 64 && kLRowDpp<T>) r[q] = lane_rot<true>(v[q]);
        else r[q] = __shfl(v[q], L.src_next, 64);
    }
    lrow_seam<T, K, 1>(r, out, L.seam_next, std::make_integer_sequence<int, K>{});
}

template <typename T, int K, int W>
__device__ __forceinline__ void lrow_prev(const T* v, T* out, const LRowLanes<W>& L)
{
    T r[K];
#pragma unroll
    for (int q = 0; q < K; q++) {
        if constexpr (W == 64 && kLRowDpp<T>) r[q] = lane_rot<false>(v[q]);
        else r[q] = __shfl(v[q], L.src_prev, 64);
    }
    lrow_seam<T, K, K - 1>(r, out, L.seam_prev, std::make_integer_sequence<int, K>{});
}

// Row offsets and flags of one lane of a lane-row wavefront; logical
// workgroup lb holds rows 4 R lb .. 4 R lb + 4 R - 1 (R = 64 / W rows per
// wavefront; with W = 64 every offset is uniform across the wavefront).
template <int W>
struct LRowSite {
    long long N, rb, rym, ryp, rzm, rzp;
    LRowLanes<W> L;
    bool live;   // lanes past the last row only join the block reduction
};

template <int W>
__device__ __forceinline__ LRowSite<W> lrow_site(const Grid& g, unsigned lb)
{
    LRowSite<W> S;
    S.L = lrow_lanes<W>();
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const unsigned nrows = (unsigned)ny * (unsigned)nz;
    constexpr unsigned R = 64u / W;
    const unsigned rw = (lb * 4u + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * R + (threadIdx.x & 63u) / W;
    S.live = rw < nrows;
    const unsigned row = S.live ? rw : 0u;
    const int j = (int)(row % (unsigned)ny), k = (int)(row / (unsigned)ny);
    const int jm = wrap_idx(j - 1, ny, g.bc), jp = wrap_idx(j + 1, ny, g.bc);
    const int km = wrap_idx(k - 1, nz, g.bc), kp = wrap_idx(k + 1, nz, g.bc);
    S.N = g.N;
    S.rb = (long long)nx * (j + (long long)ny * k);
    S.rym = (long long)nx * (jm + (long long)ny * k);
    S.ryp = (long long)nx * (jp + (long long)ny * k);
    S.rzm = (long long)nx * (j + (long long)ny * km);
    S.rzp = (long long)nx * (j + (long long)ny * kp);
    return S;
}

// EMF pipeline E of ct_x_body on a lane row (0: B_y own, 1: B_y at +y,
// 2: B_z own, 3: B_z at +z): the limited EMF G at x + 1/2 and gm at x - 1/2.
template <typename T, int K, int W, int E>
__device__ __forceinline__ void lrow_emf(const T* __restrict__ uin, const LRowSite<W>& S, T dt, const T (&r)[K],
                                         const T (&m)[K], const T (&Bk)[K], T (&G)[K], T (&gm)[K])
{
    const long long N = S.N;
    const LRowLanes<W>& L = S.L;
    const long long rn = E == 0 ? S.rym : E == 1 ? S.ryp : E == 2 ? S.rzm : S.rzp;
    T vh[K];
#pragma unroll
    for (int q = 0; q < K; q++) {
        const int x = lrow_x(L, q);
        const T r0 = r[q], m0 = m[q];
        const T rn0 = uin[rn + x], mn0 = uin[N + rn + x];
        // lower neighbour first for pencils 0 and 2, own cell first for 1 and 3
        vh[q] = (E & 1) ? qdiv(m0 + mn0, r0 + rn0) : qdiv(mn0 + m0, rn0 + r0);
    }
    T vn[K], vp[K], vv[K], qb[K];
    lrow_next<T, K, W>(vh, vn, L);
    lrow_prev<T, K, W>(vh, vp, L);
#pragma unroll
    for (int q = 0; q < K; q++) {
        vv[q] = T(0.25) * (vp[q] + T(2) * vh[q] + vn[q]);
        qb[q] = vv[q] * Bk[q];
    }
    T vvn[K], qbn[K], ev[K], g1[K];
    lrow_next<T, K, W>(vv, vvn, L);
    lrow_next<T, K, W>(qb, qbn, L);
#pragma unroll
    for (int q = 0; q < K; q++) {
        ev[q] = T(0.5) * (vv[q] + vvn[q]);
        g1[q] = ev[q] > T(0) ? qb[q] : qbn[q];
    }
    T g1p[K], qh[K];
    lrow_prev<T, K, W>(g1, g1p, L);
#pragma unroll
    for (int q = 0; q < K; q++) {
        const T bhalf = Bk[q] - (dt * T(0.5)) * (g1[q] - g1p[q]);
        qh[q] = vv[q] * bhalf;
    }
    T qhm[K], qhp[K], sq[K], sqp[K];
    lrow_prev<T, K, W>(qh, qhm, L);
    lrow_next<T, K, W>(qh, qhp, L);
#pragma unroll
    for (int q = 0; q < K; q++) sq[q] = vanleer_half(qh[q] - qhm[q], qhp[q] - qh[q]);
    lrow_next<T, K, W>(sq, sqp, L);
#pragma unroll
    for (int q = 0; q < K; q++) G[q] = ev[q] > T(0) ? qh[q] + sq[q] : qhp[q] - sqp[q];
    lrow_prev<T, K, W>(G, gm, L);
}

// Field update of ct_x_body on a lane row: from rho and m_x of the row (r, m)
// and the old faces, the new faces nB = (B_x, B_y, B_y(+y), B_z, B_z(+z)).
template <typename T, int K, int W, bool NT>
__device__ __forceinline__ void lrow_field(const T* __restrict__ uin, const T* __restrict__ bin, const LRowSite<W>& S,
                                           T dt, bool frozen, const T (&r)[K], const T (&m)[K], T (&nB)[5][K])
{
    const long long N = S.N;
    const LRowLanes<W>& L = S.L;
    T bx[K], B0[K], B1[K], B2[K], B3[K];
#pragma unroll
    for (int q = 0; q < K; q++) {
        const int x = lrow_x(L, q);
        bx[q] = ld_own<NT>(&bin[S.rb + x]);
        B0[q] = bin[N + S.rb + x];
        B1[q] = bin[N + S.ryp + x];
        B2[q] = bin[2 * N + S.rb + x];
        B3[q] = bin[2 * N + S.rzp + x];
    }
    T G0[K], g0[K], G1[K], g1[K], G2[K], g2[K], G3[K], g3[K];
    lrow_emf<T, K, W, 0>(uin, S, dt, r, m, B0, G0, g0);
    lrow_emf<T, K, W, 1>(uin, S, dt, r, m, B1, G1, g1);
    lrow_emf<T, K, W, 2>(uin, S, dt, r, m, B2, G2, g2);
    lrow_emf<T, K, W, 3>(uin, S, dt, r, m, B3, G3, g3);
    // (selects, not branches: a branch here made the compiler address these
    // arrays through a stack copy)
#pragma unroll
    for (int q = 0; q < K; q++) {
        const T n1 = B0[q] - dt * (G0[q] - g0[q]);
        const T n2 = B1[q] - dt * (G1[q] - g1[q]);
        const T n3 = B2[q] - dt * (G2[q] - g2[q]);
        const T n4 = B3[q] - dt * (G3[q] - g3[q]);
        const T n0 = (bx[q] + dt * (g1[q] - g0[q])) + dt * (g3[q] - g2[q]);
        nB[0][q] = frozen ? bx[q] : n0;
        nB[1][q] = frozen ? B0[q] : n1;
        nB[2][q] = frozen ? B1[q] : n2;
        nB[3][q] = frozen ? B2[q] : n3;
        nB[4][q] = frozen ? B3[q] : n4;
    }
}

// Logical workgroup lb holds rows 4 lb .. 4 lb + 3.
template <typename T, int K, int W, bool CFL, bool NT = true>
__device__ __forceinline__ void ct_fluid_x_lrow_body(const T* __restrict__ uin, T* __restrict__ uout,
                                                     const T* __restrict__ bin, T* __restrict__ bout,
                                                     const Grid& g, T gamma, const Ctl* __restrict__ ctl,
                                                     double dt_arg, unsigned lb,
                                                     unsigned long long* __restrict__ part)
{
    const LRowSite<W> S = lrow_site<W>(g, lb);
    const LRowLanes<W>& L = S.L;
    const bool live = S.live;   // lanes past the last row only join the block reduction
    const long long N = S.N, rb = S.rb, rym = S.rym, ryp = S.ryp, rzm = S.rzm, rzp = S.rzp;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;

    // ---- field update (as in ct_x_body), pencil by pencil
    T u[5][K], bx[K], nB[5][K], G[4][K], gm[4][K], Bk[4][K];
#pragma unroll
    for (int q = 0; q < K; q++) {
        const int x = lrow_x(L, q);
        const long long c = rb + x;
        u[0][q] = uin[c];
        u[1][q] = uin[N + c];
        u[2][q] = ld_own<NT>(&uin[2 * N + c]);
        u[3][q] = ld_own<NT>(&uin[3 * N + c]);
        u[4][q] = ld_own<NT>(&uin[4 * N + c]);
        bx[q] = ld_own<NT>(&bin[c]);
        Bk[0][q] = bin[N + c];
        Bk[1][q] = bin[N + ryp + x];
        Bk[2][q] = bin[2 * N + c];
        Bk[3][q] = bin[2 * N + rzp + x];
    }
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const long long rn = e == 0 ? rym : e == 1 ? ryp : e == 2 ? rzm : rzp;
        T vh[K];
#pragma unroll
        for (int q = 0; q < K; q++) {
            const int x = lrow_x(L, q);
            const T r0 = u[0][q], m0 = u[1][q];
            const T rn0 = uin[rn + x], mn0 = uin[N + rn + x];
            // lower neighbour first for pencils 0 and 2, own cell first for 1 and 3
            vh[q] = (e & 1) ? qdiv(m0 + mn0, r0 + rn0) : qdiv(mn0 + m0, rn0 + r0);
        }
        T vn[K], vp[K], vv[K], qb[K];
        lrow_next<T, K, W>(vh, vn, L);
        lrow_prev<T, K, W>(vh, vp, L);
#pragma unroll
        for (int q = 0; q < K; q++) {
            vv[q] = T(0.25) * (vp[q] + T(2) * vh[q] + vn[q]);
            qb[q] = vv[q] * Bk[e][q];
        }
        T vvn[K], qbn[K], ev[K], g1[K];
        lrow_next<T, K, W>(vv, vvn, L);
        lrow_next<T, K, W>(qb, qbn, L);
#pragma unroll
        for (int q = 0; q < K; q++) {
            ev[q] = T(0.5) * (vv[q] + vvn[q]);
            g1[q] = ev[q] > T(0) ? qb[q] : qbn[q];
        }
        T g1p[K], qh[K];
        lrow_prev<T, K, W>(g1, g1p, L);
#pragma unroll
        for (int q = 0; q < K; q++) {
            const T bhalf = Bk[e][q] - (dt * T(0.5)) * (g1[q] - g1p[q]);
            qh[q] = vv[q] * bhalf;
        }
        T qhm[K], qhp[K], sq[K], sqp[K];
        lrow_prev<T, K, W>(qh, qhm, L);
        lrow_next<T, K, W>(qh, qhp, L);
#pragma unroll
        for (int q = 0; q < K; q++) sq[q] = vanleer_half(qh[q] - qhm[q], qhp[q] - qh[q]);
        lrow_next<T, K, W>(sq, sqp, L);
#pragma unroll
        for (int q = 0; q < K; q++) G[e][q] = ev[q] > T(0) ? qh[q] + sq[q] : qhp[q] - sqp[q];
        lrow_prev<T, K, W>(G[e], gm[e], L);
    }
#pragma unroll
    for (int q = 0; q < K; q++) {
        if (frozen) {
            nB[0][q] = bx[q];
            nB[1][q] = Bk[0][q];
            nB[2][q] = Bk[1][q];
            nB[3][q] = Bk[2][q];
            nB[4][q] = Bk[3][q];
        } else {
            nB[1][q] = Bk[0][q] - dt * (G[0][q] - gm[0][q]);
            nB[2][q] = Bk[1][q] - dt * (G[1][q] - gm[1][q]);
            nB[3][q] = Bk[2][q] - dt * (G[2][q] - gm[2][q]);
            nB[4][q] = Bk[3][q] - dt * (G[3][q] - gm[3][q]);
            nB[0][q] = (bx[q] + dt * (gm[1][q] - gm[0][q])) + dt * (gm[3][q] - gm[2][q]);
        }
        if (live) {
            const long long c = rb + lrow_x(L, q);
            put<NT>(&bout[c], nB[0][q]);
            put<NT>(&bout[N + c], nB[1][q]);
            put<NT>(&bout[2 * N + c], nB[3][q]);
        }
    }
    // ---- fluid update (as in fluid_x_body) on the new field, set by set where no neighbour is needed
    T bxn[K];
    lrow_next<T, K, W>(nB[0], bxn, L);
    T b[3][K], rr[5][K], ll[5][K];
#pragma unroll
    for (int q = 0; q < K; q++) {
        b[0][q] = T(0.5) * (nB[0][q] + bxn[q]);
        b[1][q] = T(0.5) * (nB[1][q] + nB[2][q]);
        b[2][q] = T(0.5) * (nB[3][q] + nB[4][q]);
        T uq[5], bq[3] = {b[0][q], b[1][q], b[2][q]}, rq[5], lq[5];
#pragma unroll
        for (int m = 0; m < 5; m++) uq[m] = u[m][q];
        movers(uq, bq, gamma, rq, lq);
#pragma unroll
        for (int m = 0; m < 5; m++) {
            rr[m][q] = rq[m];
            ll[m][q] = lq[m];
        }
    }
    T f[5][K];
#pragma unroll
    for (int m = 0; m < 5; m++) {
        T lln[K];
        lrow_next<T, K, W>(ll[m], lln, L);
#pragma unroll
        for (int q = 0; q < K; q++) f[m][q] = rr[m][q] - lln[q];
    }
    T rp[5][K], lp[5][K];
    {
        T uh[5][K];
#pragma unroll
        for (int m = 0; m < 5; m++) {
            T fp_[K];
            lrow_prev<T, K, W>(f[m], fp_, L);
#pragma unroll
            for (int q = 0; q < K; q++) uh[m][q] = u[m][q] - (dt * T(0.5)) * (f[m][q] - fp_[q]);
        }
#pragma unroll
        for (int q = 0; q < K; q++) {
            T uq[5], bq[3] = {b[0][q], b[1][q], b[2][q]}, rq[5], lq[5];
#pragma unroll
            for (int m = 0; m < 5; m++) uq[m] = uh[m][q];
            movers(uq, bq, gamma, rq, lq);
#pragma unroll
            for (int m = 0; m < 5; m++) {
                rp[m][q] = rq[m];
                lp[m][q] = lq[m];
            }
        }
    }
    unsigned long long best = 0ull;
#pragma unroll
    for (int m = 0; m < 5; m++) {
        T a[K], d[K], al[K], dl[K], Rr[K], Ll[K], Lln[K], fp[K], fm[K];
        lrow_prev<T, K, W>(rp[m], a, L);
        lrow_next<T, K, W>(rp[m], d, L);
        lrow_prev<T, K, W>(lp[m], al, L);
        lrow_next<T, K, W>(lp[m], dl, L);
#pragma unroll
        for (int q = 0; q < K; q++) {
            const T c0 = rp[m][q], cl = lp[m][q];
            Rr[q] = c0 + vanleer_half(c0 - a[q], d[q] - c0);
            Ll[q] = cl - vanleer_half(cl - al[q], dl[q] - cl);
        }
        lrow_next<T, K, W>(Ll, Lln, L);
#pragma unroll
        for (int q = 0; q < K; q++) fp[q] = Rr[q] - Lln[q];
        lrow_prev<T, K, W>(fp, fm, L);
#pragma unroll
        for (int q = 0; q < K; q++) {
            // the new state overwrites u (its old value is not needed any more)
            u[m][q] = frozen ? u[m][q] : u[m][q] - dt * (fp[q] - fm[q]);
            if (live) put<NT>(&uout[m * N + rb + lrow_x(L, q)], u[m][q]);
        }
    }
    if constexpr (CFL) {
#pragma unroll
        for (int q = 0; q < K; q++) {
            const T cc = cfl_speed(u[0][q], u[1][q], u[2][q], u[3][q], u[4][q], b[0][q], b[1][q], b[2][q], gamma);
            const unsigned long long bits = live ? speed_bits(cc) : 0ull;
            best = bits > best ? bits : best;
        }
        block_max_to_part<256>(best, threadIdx.x, part);
    }
}

template <typename T, int K, int W, bool CFL, bool NT>
__global__ void __launch_bounds__(256) ct_fluid_x_lrow(const T* __restrict__ uin, T* __restrict__ uout,
                                                       const T* __restrict__ bin, T* __restrict__ bout, Grid g,
                                                       T gamma, const Ctl* __restrict__ ctl, double dt_arg,
                                                       unsigned long long* __restrict__ parts, int* count)
{
    if constexpr (CFL) store_part_count(count);
    ct_fluid_x_lrow_body<T, K, W, CFL, NT>(uin, uout, bin, bout, g, gamma, ctl, dt_arg, blockIdx.x,
                                       parts + blockIdx.x);
}

// B_{y->x}, B_{z->x} alone on a lane row (as ct_x_body); logical workgroup
// lb holds rows 4 lb .. 4 lb + 3.
template <typename T, int K, int W, bool NT = true>
__device__ __forceinline__ void ct_x_lrow_body(const T* __restrict__ uf, const T* __restrict__ bin,
                                               T* __restrict__ bout, const Grid& g, const Ctl* __restrict__ ctl,
                                               double dt_arg, unsigned lb)
{
    const LRowSite<W> S = lrow_site<W>(g, lb);
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;
    T r[K], m[K], nB[5][K];
#pragma unroll
    for (int q = 0; q < K; q++) {
        const long long c = S.rb + lrow_x(S.L, q);
        r[q] = uf[c];
        m[q] = uf[S.N + c];
    }
    lrow_field<T, K, W, NT>(uf, bin, S, dt, frozen, r, m, nB);
    if (S.live) {
#pragma unroll
        for (int q = 0; q < K; q++) {
            const long long c = S.rb + lrow_x(S.L, q);
            put<NT>(&bout[c], nB[0][q]);
            put<NT>(&bout[S.N + c], nB[1][q]);
            put<NT>(&bout[2 * S.N + c], nB[3][q]);
        }
    }
}

template <typename T, int K, int W, bool NT>
__global__ void __launch_bounds__(256) ct_x_lrow(const T* __restrict__ uf, const T* __restrict__ bin,
                                                 T* __restrict__ bout, Grid g, const Ctl* __restrict__ ctl,
                                                 double dt_arg)
{
    ct_x_lrow_body<T, K, W, NT>(uf, bin, bout, g, ctl, dt_arg, blockIdx.x);
}

// fluid_x alone on a lane row (as fluid_x_body), in FP32: plain handles on
// every row length the form takes, batches on rows of 32 to 128 cells, where
// the wavefront form wastes a quarter to a half of its lanes.
// With CFL the rows' largest CFL speed goes to part (all threads take part).
template <typename T, int K, int W, bool CFL, bool NT = true>
__device__ __forceinline__ void fluid_x_lrow_body(const T* __restrict__ uin, T* __restrict__ uout,
                                                  const T* __restrict__ bf, const Grid& g, T gamma,
                                                  const Ctl* __restrict__ ctl, double dt_arg, unsigned lb,
                                                  unsigned long long* __restrict__ part)
{
    const LRowSite<W> S = lrow_site<W>(g, lb);
    const long long N = S.N;
    const LRowLanes<W>& L = S.L;
    const T dt = (T)(dt_arg >= 0.0 ? dt_arg : ctl->dt);
    const bool frozen = ctl->status != 0;
    T u[5][K], b[3][K], bx[K], bxn[K];
#pragma unroll
    for (int q = 0; q < K; q++) {
        const int x = lrow_x(L, q);
        const long long c = S.rb + x;
#pragma unroll
        for (int m = 0; m < 5; m++) u[m][q] = ld_own<NT>(&uin[m * N + c]);
        bx[q] = ld_own<NT>(&bf[c]);
        b[1][q] = T(0.5) * (bf[N + c] + bf[N + S.ryp + x]);
        b[2][q] = T(0.5) * (bf[2 * N + c] + bf[2 * N + S.rzp + x]);
    }
    lrow_next<T, K, W>(bx, bxn, L);
#pragma unroll
    for (int q = 0; q < K; q++) b[0][q] = T(0.5) * (bx[q] + bxn[q]);
    T rr[5][K], ll[5][K];
#pragma unroll
    for (int q = 0; q < K; q++) {
        T uq[5], bq[3] = {b[0][q], b[1][q], b[2][q]}, rq[5], lq[5];
#pragma unroll
        for (int m = 0; m < 5; m++) uq[m] = u[m][q];
        movers(uq, bq, gamma, rq, lq);
#pragma unroll
        for (int m = 0; m < 5; m++) {
            rr[m][q] = rq[m];
            ll[m][q] = lq[m];
        }
    }
    T f[5][K];
#pragma unroll
    for (int m = 0; m < 5; m++) {
        T lln[K];
        lrow_next<T, K, W>(ll[m], lln, L);
#pragma unroll
        for (int q = 0; q < K; q++) f[m][q] = rr[m][q] - lln[q];
    }
    T rp[5][K], lp[5][K];
    {
        T uh[5][K];
#pragma unroll
        for (int m = 0; m < 5; m++) {
            T fp_[K];
            lrow_prev<T, K, W>(f[m], fp_, L);
#pragma unroll
            for (int q = 0; q < K; q++) uh[m][q] = u[m][q] - (dt * T(0.5)) * (f[m][q] - fp_[q]);
        }
#pragma unroll
        for (int q = 0; q < K; q++) {
            T uq[5], bq[3] = {b[0][q], b[1][q], b[2][q]}, rq[5], lq[5];
#pragma unroll
            for (int m = 0; m < 5; m++) uq[m] = uh[m][q];
            movers(uq, bq, gamma, rq, lq);
#pragma unroll
            for (int m = 0; m < 5; m++) {
                rp[m][q] = rq[m];
                lp[m][q] = lq[m];
            }
        }
    }
#pragma unroll
    for (int m = 0; m < 5; m++) {
        T a[K], d[K], al[K], dl[K], Rr[K], Ll[K], Lln[K], fp[K], fm[K];
        lrow_prev<T, K, W>(rp[m], a, L);
        lrow_next<T, K, W>(rp[m], d, L);
        lrow_prev<T, K, W>(lp[m], al, L);
        lrow_next<T, K, W>(lp[m], dl, L);
#pragma unroll
        for (int q = 0; q < K; q++) {
            const T c0 = rp[m][q], cl = lp[m][q];
            Rr[q] = c0 + vanleer_half(c0 - a[q], d[q] - c0);
            Ll[q] = cl - vanleer_half(cl - al[q], dl[q] - cl);
        }
        lrow_next<T, K, W>(Ll, Lln, L);
#pragma unroll
        for (int q = 0; q < K; q++) fp[q] = Rr[q] - Lln[q];
        lrow_prev<T, K, W>(fp, fm, L);
#pragma unroll
        for (int q = 0; q < K; q++) {
            u[m][q] = frozen ? u[m][q] : u[m][q] - dt * (fp[q] - fm[q]);
            if (S.live) put<NT>(&uout[m * N + S.rb + lrow_x(L, q)], u[m][q]);
        }
    }
    if constexpr (CFL) {
        unsigned long long best = 0ull;
#pragma unroll
        for (int q = 0; q < K; q++) {
            const T cc = cfl_speed(u[0][q], u[1][q], u[2][q], u[3][q], u[4][q], b[0][q], b[1][q], b[2][q], gamma);
            const unsigned long long bits = S.live ? speed_bits(cc) : 0ull;
            best = bits > best ? bits : best;
        }
        block_max_to_part<256>(best, threadIdx.x, part);
    }
}

template <typename T, int K, int W, bool CFL, bool NT>
__global__ void __launch_bounds__(256) fluid_x_lrow(const T* __restrict__ uin, T* __restrict__ uout,
                                                    const T* __restrict__ bf, Grid g, T gamma,
                                                    const Ctl* __restrict__ ctl, double dt_arg,
                                                    unsigned long long* __restrict__ parts, int* count)
{
    if constexpr (CFL) store_part_count(count);
    fluid_x_lrow_body<T, K, W, CFL, NT>(uin, uout, bf, g, gamma, ctl, dt_arg, blockIdx.x, parts + blockIdx.x);
}

// Shape of the lane-row form on a periodic grid: W lanes per row and K cells
// per lane, rows of W K cells (returns K, 0 where the form does not apply):
// rows of 64, 128, 192 or 256 cells fill a wavefront each (W = 64, K = 1-4);
// rows of 32 and 96 cells share one two at a time (W = 32, K = 1 or 3), rows
// of 48 four at a time (W = 16, K = 3). Rows of other lengths run the
// wavefront form. The field update along x takes the form in both precisions
// (FP64 256^3: 0.303 -> 0.254 ms against the wavefront form); the fluid update
// and the fused reverse L_x take it in FP32 only: FP64 periodic rows of 64 k
// cells run both in the row-per-workgroup form (the FP64 fluid update in the
// lane-row form measured 0.379 ms, in the row form 0.302; the fused sweep
// needs 247-256 VGPRs in the lane-row form).
static int x_lrow_k(const Grid& g, int* W, int kmax = 4)
{
    if (g.bc != 0) return 0;
    const int n = g.n[0];
    int w = 0, k = 0;
    if (n % 64 == 0 && n <= 256) {
        w = 64;
        k = n / 64;
    } else if (n == 32 || n == 96) {
        w = 32;
        k = n / 32;
    } else if (n == 48) {
        w = 16;
        k = 3;
    }
    if (k == 0 || k > kmax) return 0;
    *W = w;
    return k;
}

// Calls X(K, W) for the (K, W) of the grid's lane-row shape.
#define MHD_LROW_DISPATCH(K, W, X)                 \
    switch ((K) * 100 + (W)) {                     \
    case 164: X(1, 64) break;                      \
    case 264: X(2, 64) break;                      \
    case 364: X(3, 64) break;                      \
    case 464: X(4, 64) break;                      \
    case 132: X(1, 32) break;                      \
    case 332: X(3, 32) break;                      \
    default: X(3, 16) break;                       \
    }

template <typename T>
static int x_lrow_k_fluid(const Grid& g, int* W)
{
    return kExact<T> ? 0 : x_lrow_k(g, W);
}

// Workgroups of a lane-row launch: four wavefronts of 64 / W rows each.
static unsigned x_lrow_blocks(const Grid& g, int W)
{
    const long long rows_per_block = 4LL * (64 / W);
    return (unsigned)(((long long)g.n[1] * g.n[2] + rows_per_block - 1) / rows_per_block);
}

// ---------------------------------------------------------------------------
constexpr int RB = 256;   // threads per block of the reductions

// Per-cell CFL speed of eq. equat_CFL; per-block maxima into parts.
template <typename T>
__device__ __forceinline__ void cfl_body(const T* __restrict__ u, const T* __restrict__ b, const Grid& g, T gamma,
                                         unsigned lb, unsigned nb, unsigned long long* __restrict__ part)
{
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const long long N = g.N;
    unsigned long long best = 0ull;
    // one x-row (j, k) per loop trip of a block, lanes along x
    const long long nrows = (long long)ny * nz;
    for (long long row = lb; row < nrows; row += nb) {
        const int j = (int)(row % ny), k = (int)(row / ny);
        const long long rb = row * nx;
        const long long yoff = (long long)(wrap_idx(j + 1, ny, g.bc) - j) * nx;
        const long long zoff = (long long)(wrap_idx(k + 1, nz, g.bc) - k) * nx * ny;
        for (int i = threadIdx.x; i < nx; i += RB) {
            const long long c = rb + i;
            const long long cxp = rb + wrap_idx(i + 1, nx, g.bc);
            const T bx = T(0.5) * (b[c] + b[cxp]);
            const T by = T(0.5) * (b[N + c] + b[N + c + yoff]);
            const T bz = T(0.5) * (b[2 * N + c] + b[2 * N + c + zoff]);
            const T cc = cfl_speed(u[c], u[N + c], u[2 * N + c], u[3 * N + c], u[4 * N + c], bx, by, bz, gamma);
            const unsigned long long bits = speed_bits(cc);
            best = bits > best ? bits : best;
        }
    }
    block_max_to_part<RB>(best, threadIdx.x, part);
}

template <typename T>
__global__ void __launch_bounds__(RB) cfl_kernel(const T* __restrict__ u, const T* __restrict__ b, Grid g,
                                                 T gamma, unsigned long long* __restrict__ parts, int* count)
{
    store_part_count(count);
    cfl_body<T>(u, b, g, gamma, blockIdx.x, gridDim.x, parts + blockIdx.x);
}

// max over cells of |div B| (cells whose upper faces are stored)
template <typename T>
__global__ void __launch_bounds__(RB) divb_kernel(const T* __restrict__ b, Grid g,
                                                  unsigned long long* __restrict__ parts)
{
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const long long N = g.N;
    unsigned long long best = 0ull;
    const long long nrows = (long long)ny * nz;
    for (long long row = blockIdx.x; row < nrows; row += gridDim.x) {
      const int j = (int)(row % ny), k = (int)(row / ny);
      if (g.bc != 0 && ((ny > 1 && j == ny - 1) || (nz > 1 && k == nz - 1))) continue;
      const long long rb = row * nx;
      const long long yoff = (long long)(wrap_idx(j + 1, ny, g.bc) - j) * nx;
      const long long zoff = (long long)(wrap_idx(k + 1, nz, g.bc) - k) * nx * ny;
      for (int i = threadIdx.x; i < nx; i += RB) {
        if (g.bc != 0 && nx > 1 && i == nx - 1) continue;
        const long long c = rb + i;
        const long long cxp = rb + wrap_idx(i + 1, nx, g.bc);
        const long long cyp = c + yoff;
        const long long czp = c + zoff;
        double d = (double)(b[cxp] - b[c]);
        d += (double)(b[N + cyp] - b[N + c]);
        d += (double)(b[2 * N + czp] - b[2 * N + c]);
        const unsigned long long bits = speed_bits(fabs(d));
        best = bits > best ? bits : best;
      }
    }
    block_max_to_part<RB>(best, threadIdx.x, parts + blockIdx.x);
}

int reduce_blocks(const Grid& g)
{
    // one block per x-row (several rows per block on large grids)
    long long b = (long long)g.n[1] * g.n[2];
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return (int)b;
}

// chunk length along the sweep for the marching kernels: about `target`
// wavefronts in all (enough to fill the device), but no shorter than four
// ghost depths, where the warm-up (two ghost depths per chunk) would cost
// half the work. Mid-size and 2D grids need the short chunks to fill the
// device (128^3 blast step 24-31 % faster, Orszag-Tang 512^2 37 %, than
// with a floor of sixteen ghost depths); 256^3 takes 128-cell chunks. With
// `fill` (a launch that has the device to itself) a grid that would still
// give fewer than target / 2 wavefronts goes down to two ghost depths: the
// doubled warm-up costs less than the idle device (Orszag-Tang 512^2 17 %
// faster); a batch fills the device with other problems and keeps four.
int march_chunk(const Grid& g, int d, int ghost, long long target, bool fill = false)
{
    const int ta = (d == 1) ? 2 : 1;
    const long long waves = march_packed(g.n[0]) ? ((long long)g.n[0] * g.n[ta] + 63) / 64
                                                 : ((g.n[0] + 63) / 64) * (long long)g.n[ta];
    const int nd = g.n[d];
    long long want = target / (waves > 0 ? waves : 1);
    if (want < 1) want = 1;
    int chunk = (int)((nd + want - 1) / want);
    int minchunk = 4 * ghost;
    if (fill && waves * ((nd + minchunk - 1) / minchunk) < target / 2) minchunk = 2 * ghost;
    if (chunk < minchunk) chunk = minchunk;
    if (chunk > nd) chunk = nd;
    return chunk;
}

}  // namespace

static unsigned march_blocks(const Grid& g, int axis, int chunk, bool xwide)
{
    const int ta = (axis == 1) ? 2 : 1;
    if (march_packed(g.n[0])) {
        const long long P = (long long)g.n[0] * g.n[ta];
        return (unsigned)(((P + 64 * MW - 1) / (64 * MW)) * ((g.n[axis] + chunk - 1) / chunk));
    }
    const int wx = march_wx(axis, g.n[0], g.n[ta], xwide), wt = MW / wx;
    return (unsigned)(((g.n[0] + 64 * wx - 1) / (64 * wx)) * ((g.n[ta] + wt - 1) / wt) *
                      ((g.n[axis] + chunk - 1) / chunk));
}

template <typename T>
hipError_t launch_cfl(const T* u, const T* b, Grid g, double gamma, unsigned long long* parts, Ctl* ctl,
                      hipStream_t s)
{
    const int nb = reduce_blocks(g);
    hipLaunchKernelGGL((cfl_kernel<T>), dim3(nb), dim3(RB), 0, s, u, b, g, (T)gamma, parts, &ctl->nparts);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_divb(const T* b, Grid g, unsigned long long* parts, int* nparts, hipStream_t s)
{
    const int nb = reduce_blocks(g);
    hipLaunchKernelGGL((divb_kernel<T>), dim3(nb), dim3(RB), 0, s, b, g, parts);
    *nparts = nb;
    return hipGetLastError();
}

// Cache policy of a sweep's output stores and read-once loads (see put):
// non-temporal where the state is larger than about two thirds of the 256 MB
// memory-side last-level cache, plain where the next sweep still finds much
// of the state there. Step times of the blast, plain / non-temporal: 128^3
// (128 MiB FP64) 0.549 / 0.618 ms FP64, 0.303 / 0.325 ms FP32; 192^3 (216 MiB
// FP32) 1.971 / 1.943 ms FP64, 0.930 / 0.904 ms FP32; 256^3 3.393 / 3.313 ms
// FP64, 1.718 / 1.635 ms FP32.
constexpr long long kNtStateBytes = 160ll << 20;

template <typename T>
bool nt_policy(const Grid& g)
{
    return 8 * g.N * (long long)sizeof(T) > kNtStateBytes;
}

template <typename T, bool CFL, bool NT>
static void fluid_launch(int axis, const T* u_in, T* u_out, const T* b, Grid g, double gamma, Ctl* ctl,
                         double dt, unsigned long long* parts, hipStream_t s)
{
    int* count = CFL ? &ctl->nparts : nullptr;
    int W = 64;
    const int K = axis == 0 ? x_lrow_k_fluid<T>(g, &W) : 0;
    if (K) {
        const unsigned nb = x_lrow_blocks(g, W);
#define MHD_LROW_FLUID(KK, WW)                                                                                \
    hipLaunchKernelGGL((fluid_x_lrow<T, KK, WW, CFL, NT>), dim3(nb), dim3(256), 0, s, u_in, u_out, b, g, (T)gamma, ctl, \
                       dt, parts, count);
        MHD_LROW_DISPATCH(K, W, MHD_LROW_FLUID)
#undef MHD_LROW_FLUID
    } else if (axis == 0 && ct_fluid_x_row_ok<T>(g)) {
        hipLaunchKernelGGL((fluid_x_row<T, CFL, NT>), dim3((unsigned)((long long)g.n[1] * g.n[2])),
                           dim3(64 * (g.n[0] / 64)), 0, s, u_in, u_out, b, g, (T)gamma, ctl, dt, parts, count);
    } else if (axis == 0) {
        const unsigned nb = x_wave_blocks(g);
        hipLaunchKernelGGL((fluid_x_wave<T, CFL, NT>), dim3(nb), dim3(256), 0, s, u_in, u_out, b, g, (T)gamma, ctl, dt,
                           parts, count);
    } else {
        const int chunk = march_chunk(g, axis, GF, kFluidMarchWaves, true);
        const unsigned nb = march_blocks(g, axis, chunk, kMarchXWide<T, false>);
        const dim3 block(64, MW);
        if (axis == 1)
            hipLaunchKernelGGL((fluid_march<T, 1, CFL, NT>), dim3(nb), block, 0, s, u_in, u_out, b, g, (T)gamma, ctl, dt,
                               chunk, parts, count);
        else
            hipLaunchKernelGGL((fluid_march<T, 2, CFL, NT>), dim3(nb), block, 0, s, u_in, u_out, b, g, (T)gamma, ctl, dt,
                               chunk, parts, count);
    }
}

template <typename T>
hipError_t launch_fluid(int axis, const T* u_in, T* u_out, const T* b, Grid g, double gamma, Ctl* ctl,
                        double dt, unsigned long long* parts, hipStream_t s)
{
    const bool nt = nt_policy<T>(g);
    if (parts && nt)
        fluid_launch<T, true, true>(axis, u_in, u_out, b, g, gamma, ctl, dt, parts, s);
    else if (parts)
        fluid_launch<T, true, false>(axis, u_in, u_out, b, g, gamma, ctl, dt, parts, s);
    else if (nt)
        fluid_launch<T, false, true>(axis, u_in, u_out, b, g, gamma, ctl, dt, nullptr, s);
    else
        fluid_launch<T, false, false>(axis, u_in, u_out, b, g, gamma, ctl, dt, nullptr, s);
    return hipGetLastError();
}

// Wavefronts per fused (field + fluid) march launch: the FP64 march runs one
// wavefront per SIMD (its pipelines need every register), so one wavefront per
// SIMD in a single round (256-cell chunks at 256^3; 4 % faster than two
// rounds of 128-cell chunks); FP32 runs two per SIMD.
template <typename T>
constexpr long long kFusedMarchWaves = kExact<T> ? 1024 : 2048;

template <typename T>
static int fused_chunk(const Grid& g, int axis)
{
    return march_chunk(g, axis, GCF, kFusedMarchWaves<T>, true);
}

// The fused march pays where its chunks are long: its warm-up is 15 cells per
// chunk (against 6 and 8 for the two marches, which also run at higher
// occupancy), so grids that need short chunks to fill the device (2D planes,
// 128^3) run the two launches: measured fused / two launches per reverse
// L_y in FP64 on Orszag-Tang 512^2 0.062 / 0.041 ms, 128^3 0.105 / 0.092 ms,
// 256^3 0.565 / 0.660 ms. The fused x sweep pays on every grid.
template <typename T>
bool fused_reverse_pays(const Grid& g, int axis)
{
    return axis == 0 || fused_chunk<T>(g, axis) >= 64;
}

template <typename T, bool NT>
static hipError_t ct_fluid_launch(int axis, const T* u_in, T* u_out, const T* b_in, T* b_out, Grid g, double gamma,
                           Ctl* ctl, double dt, unsigned long long* parts, hipStream_t s)
{
    if (axis < 0 || axis > 2 || g.bc != 0) return hipErrorInvalidValue;
    int W = 64;
    const int K = axis == 0 ? x_lrow_k_fluid<T>(g, &W) : 0;
    if (K) {
        const unsigned nb = x_lrow_blocks(g, W);
#define MHD_LROW_FUSED(KK, WW)                                                                                \
    if (parts)                                                                                                \
        hipLaunchKernelGGL((ct_fluid_x_lrow<T, KK, WW, true, NT>), dim3(nb), dim3(256), 0, s, u_in, u_out, b_in, b_out, \
                           g, (T)gamma, ctl, dt, parts, &ctl->nparts);                                        \
    else                                                                                                      \
        hipLaunchKernelGGL((ct_fluid_x_lrow<T, KK, WW, false, NT>), dim3(nb), dim3(256), 0, s, u_in, u_out, b_in,      \
                           b_out, g, (T)gamma, ctl, dt, nullptr, nullptr);
        MHD_LROW_DISPATCH(K, W, MHD_LROW_FUSED)
#undef MHD_LROW_FUSED
        return hipGetLastError();
    }
    if (axis == 0 && ct_fluid_x_row_ok<T>(g)) {
        const unsigned nb = (unsigned)((long long)g.n[1] * g.n[2]);
        const dim3 block(64 * (g.n[0] / 64));
        if (parts)
            hipLaunchKernelGGL((ct_fluid_x_row<T, true, NT>), dim3(nb), block, 0, s, u_in, u_out, b_in, b_out, g,
                               (T)gamma, ctl, dt, parts, &ctl->nparts);
        else
            hipLaunchKernelGGL((ct_fluid_x_row<T, false, NT>), dim3(nb), block, 0, s, u_in, u_out, b_in, b_out, g,
                               (T)gamma, ctl, dt, nullptr, nullptr);
        return hipGetLastError();
    }
    if (axis == 0) {
        const unsigned nb = ct_fluid_x_blocks(g);
        if (parts)
            hipLaunchKernelGGL((ct_fluid_x_wave<T, true, NT>), dim3(nb), dim3(256), 0, s, u_in, u_out, b_in, b_out, g,
                               (T)gamma, ctl, dt, parts, &ctl->nparts);
        else
            hipLaunchKernelGGL((ct_fluid_x_wave<T, false, NT>), dim3(nb), dim3(256), 0, s, u_in, u_out, b_in, b_out, g,
                               (T)gamma, ctl, dt, nullptr, nullptr);
        return hipGetLastError();
    }
    const int chunk = fused_chunk<T>(g, axis);
    const dim3 grid(march_blocks(g, axis, chunk, kMarchXWide<T, true>)), block(64, MW);
    if (parts) {
        if (axis == 1)
            hipLaunchKernelGGL((ct_fluid_march<T, 1, true, NT>), grid, block, 0, s, u_in, u_out, b_in, b_out, g, (T)gamma,
                               ctl, dt, chunk, parts, &ctl->nparts);
        else
            hipLaunchKernelGGL((ct_fluid_march<T, 2, true, NT>), grid, block, 0, s, u_in, u_out, b_in, b_out, g, (T)gamma,
                               ctl, dt, chunk, parts, &ctl->nparts);
    } else {
        if (axis == 1)
            hipLaunchKernelGGL((ct_fluid_march<T, 1, false, NT>), grid, block, 0, s, u_in, u_out, b_in, b_out, g,
                               (T)gamma, ctl, dt, chunk, nullptr, nullptr);
        else
            hipLaunchKernelGGL((ct_fluid_march<T, 2, false, NT>), grid, block, 0, s, u_in, u_out, b_in, b_out, g,
                               (T)gamma, ctl, dt, chunk, nullptr, nullptr);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ct_fluid(int axis, const T* u_in, T* u_out, const T* b_in, T* b_out, Grid g, double gamma,
                           Ctl* ctl, double dt, unsigned long long* parts, hipStream_t s)
{
    if (nt_policy<T>(g)) return ct_fluid_launch<T, true>(axis, u_in, u_out, b_in, b_out, g, gamma, ctl, dt, parts, s);
    return ct_fluid_launch<T, false>(axis, u_in, u_out, b_in, b_out, g, gamma, ctl, dt, parts, s);
}

template <typename T, bool NT>
static hipError_t ct_launch(int axis, const T* u, const T* b_in, T* b_out, Grid g, const Ctl* ctl, double dt,
                     hipStream_t s)
{
    int W = 64;
    const int K = axis == 0 ? x_lrow_k(g, &W) : 0;
    if (K) {
        const unsigned nb = x_lrow_blocks(g, W);
#define MHD_LROW_CT(KK, WW) \
    hipLaunchKernelGGL((ct_x_lrow<T, KK, WW, NT>), dim3(nb), dim3(256), 0, s, u, b_in, b_out, g, ctl, dt);
        MHD_LROW_DISPATCH(K, W, MHD_LROW_CT)
#undef MHD_LROW_CT
    } else if (axis == 0) {
        hipLaunchKernelGGL((ct_x_wave<T, NT>), dim3(ct_x_wave_blocks(g)), dim3(256), 0, s, u, b_in, b_out, g, ctl, dt);
    } else {
        const int chunk = march_chunk(g, axis, GB, kCtMarchWaves<T>, true);
        const dim3 grid(march_blocks(g, axis, chunk, kMarchXWide<T, true>)), block(64, MW);
        if (axis == 1)
            hipLaunchKernelGGL((ct_march<T, 1, NT>), grid, block, 0, s, u, b_in, b_out, g, ctl, dt, chunk);
        else
            hipLaunchKernelGGL((ct_march<T, 2, NT>), grid, block, 0, s, u, b_in, b_out, g, ctl, dt, chunk);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ct(int axis, const T* u, const T* b_in, T* b_out, Grid g, const Ctl* ctl, double dt,
                     hipStream_t s)
{
    if (nt_policy<T>(g)) return ct_launch<T, true>(axis, u, b_in, b_out, g, ctl, dt, s);
    return ct_launch<T, false>(axis, u, b_in, b_out, g, ctl, dt, s);
}

}  // namespace mhd

"""Seeded synthetic initial states for the MHD step (numpy only).

These generators build the test problems of Wong et al. (Sec. 5: Brio-Wu shock
tube, Orszag-Tang vortex, blast waves) and smooth states for checking the
solver (linear MHD waves with closed-form solutions, random smooth states).
They only sample initial conditions; none of the solver's arithmetic lives
here. Both the oracle and the GPU library consume these states.

Conventions: cells are cubes of width h = 1 / max(nx, ny, nz) (the solver
works in unit cells), so the box is [0, nx h) x [0, ny h) x [0, nz h); periodic
patterns use whole periods of each box side. A state is a float64 array of shape (8, nz, ny, nx) holding
rho, m_x, m_y, m_z, E, B_x, B_y, B_z with x fastest. B_d is sampled on the
lower d-face of each cell (Sec. 3, eq. equat_b). Where the field is not
constant along its own axis it is built as the discrete curl of an edge vector
potential, so its discrete divergence vanishes to round-off. The total energy
uses the analytic field at the cell centre. In code units (unit cells) a
physical time t is t / h.
"""
from __future__ import annotations

import math

import numpy as np

MASTER_SEED = 9084362


def cell_width(nx, ny, nz):
    return 1.0 / max(nx, ny, nz)


def _centres(n, h):
    return (np.arange(n) + 0.5) * h


def _faces(n, h):
    return np.arange(n) * h


def _grid(nx, ny, nz, kind):
    """Coordinates (x, y, z) broadcastable to (nz, ny, nx); kind gives, per axis,
    'c' for cell centres or 'f' for lower faces."""
    h = cell_width(nx, ny, nz)
    ax = []
    for n, k in zip((nx, ny, nz), kind):
        ax.append(_centres(n, h) if k == "c" else _faces(n, h))
    x = ax[0][None, None, :]
    y = ax[1][None, :, None]
    z = ax[2][:, None, None]
    return x, y, z


def assemble(rho, vel, p, bface, bcentre, gamma, shape):
    """State array from primitive cell values, face fields and centred field.

    rho, p: cell values; vel, bcentre: 3-tuples of cell values; bface: 3-tuple
    of face values (each broadcastable to shape = (nz, ny, nx)).
    """
    nz, ny, nx = shape
    s = np.zeros((8, nz, ny, nx), dtype=np.float64)
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), shape)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), shape)
    v = [np.broadcast_to(np.asarray(c, dtype=np.float64), shape) for c in vel]
    bc = [np.broadcast_to(np.asarray(c, dtype=np.float64), shape) for c in bcentre]
    s[0] = rho
    for a in range(3):
        s[1 + a] = rho * v[a]
        s[5 + a] = np.broadcast_to(np.asarray(bface[a], dtype=np.float64), shape)
    kin = 0.5 * rho * (v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    mag = 0.5 * (bc[0] ** 2 + bc[1] ** 2 + bc[2] ** 2)
    s[4] = p / (gamma - 1.0) + kin + mag
    return s


def curl_faces(ax_fn, ay_fn, az_fn, nx, ny, nz):
    """Face fields of the discrete curl of an edge vector potential.

    a_x lives on x-edges (cell-centre x, face y, face z), a_y on y-edges and a_z
    on z-edges. Each *_fn(x, y, z) is evaluated on the needed edge points
    (periodic potentials). Differences are taken over one cell (width h)."""
    h = cell_width(nx, ny, nz)

    def ev(fn, x, y, z):
        return np.broadcast_to(fn(x, y, z), (nz, ny, nx)).astype(np.float64)

    xc, yc, zc = _grid(nx, ny, nz, "ccc")
    xf, yf, zf = _grid(nx, ny, nz, "fff")
    bx = (ev(az_fn, xf, yf + h, zc) - ev(az_fn, xf, yf, zc)) / h - (
        ev(ay_fn, xf, yc, zf + h) - ev(ay_fn, xf, yc, zf)) / h
    by = (ev(ax_fn, xc, yf, zf + h) - ev(ax_fn, xc, yf, zf)) / h - (
        ev(az_fn, xf + h, yf, zc) - ev(az_fn, xf, yf, zc)) / h
    bz = (ev(ay_fn, xf + h, yc, zf) - ev(ay_fn, xf, yc, zf)) / h - (
        ev(ax_fn, xc, yf + h, zf) - ev(ax_fn, xc, yf, zf)) / h
    return bx, by, bz


# --------------------------------------------------------------------------
# Problems of the paper (Sec. 5)
# --------------------------------------------------------------------------

def brio_wu(n: int, gamma: float = 2.0, axis: int = 0, ntrans: int = 1):
    """Brio-Wu shock tube (Sec. 5.1.1) laid along `axis` (n cells), interface at
    0.5 (cell centres below 0.5 take the left state); the normal field is 0.75
    and the first transverse field +1 / -1. Transverse axes have ntrans cells."""
    shape_xyz = [ntrans, ntrans, ntrans]
    shape_xyz[axis] = n
    nx, ny, nz = shape_xyz
    shape = (nz, ny, nx)
    pos = (np.arange(n) + 0.5) / n
    left = pos < 0.5
    sel = [None, None, None]
    sel[2 - axis] = slice(None)
    L = left[tuple(sel)]
    rho = np.where(L, 1.0, 0.125)
    p = np.where(L, 1.0, 0.1)
    t1 = (axis + 1) % 3
    bvals = [0.0, 0.0, 0.0]
    bvals[axis] = 0.75
    bt = np.where(L, 1.0, -1.0)
    bcomp = [np.zeros(shape) + bvals[a] for a in range(3)]
    bcomp[t1] = np.broadcast_to(bt, shape).astype(np.float64)
    return assemble(rho, (0.0, 0.0, 0.0), p, bcomp, bcomp, gamma, shape)


def orszag_tang(n: int, nz: int = 1, gamma: float = 5.0 / 3.0):
    """Orszag-Tang vortex (Sec. 5.2.1) on n x n (x nz, extruded along z)."""
    b0 = 1.0 / math.sqrt(4.0 * math.pi)
    shape = (nz, n, n)
    xc, yc, _ = _grid(n, n, nz, "ccc")
    rho = 25.0 / (36.0 * math.pi)
    p = 5.0 / (12.0 * math.pi)
    vx = -np.sin(2 * math.pi * yc)
    vy = np.sin(2 * math.pi * xc)
    # B_x on x-faces depends on y only, B_y on y-faces on x only: the face values
    # equal the centre values and the field is exactly divergence free.
    bx = -b0 * np.sin(2 * math.pi * yc) + 0.0 * xc
    by = b0 * np.sin(4 * math.pi * xc) + 0.0 * yc
    bz = np.zeros(shape)
    return assemble(rho, (vx, vy, 0.0), p, (bx, by, bz), (bx, by, bz), gamma, shape)


def blast(n: int, p_in: float = 10.0, p_out: float = 0.1, radius: float = 0.1,
          bvec=(1.0 / math.sqrt(2.0), 1.0 / math.sqrt(2.0), 0.0), gamma: float = 5.0 / 3.0,
          ny: int | None = None, nz: int | None = None, centre=(0.5, 0.5, 0.5)):
    """Blast wave (Sec. 5.2.2, 5.3): rho = 1, v = 0, uniform B, p = p_in for cell
    centres strictly inside the sphere, p_out elsewhere."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    shape = (nz, ny, n)
    x, y, z = _grid(n, ny, nz, "ccc")
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2
    if nz > 1:
        r2 = r2 + (z - centre[2]) ** 2
    p = np.where(r2 < radius * radius, p_in, p_out)
    b = tuple(np.full(shape, float(c)) for c in bvec)
    return assemble(1.0, (0.0, 0.0, 0.0), p, b, b, gamma, shape)


def dai_woodward(n: int, axis: int = 0, ntrans: int = 1, gamma: float = 5.0 / 3.0):
    """MHD shock tube of Sec. 5.1.2 (Dai and Woodward) along `axis`: left
    (cell centre < 0.5) rho 1.08, p 0.95, v = (1.2, 0.01, 0.5), B = (2, 3.6, 2)
    / sqrt(4 pi); right rho 1, p 1, v = 0, B = (2, 4, 2) / sqrt(4 pi). The
    normal field is read as 2 / sqrt(4 pi), like the transverse ones (the
    printed 2 sqrt(4 pi) is taken as a typo). Components are given along the
    tube (normal first, then the two transverse axes in cyclic order)."""
    shape_xyz = [ntrans, ntrans, ntrans]
    shape_xyz[axis] = n
    nx, ny, nz = shape_xyz
    shape = (nz, ny, nx)
    pos = (np.arange(n) + 0.5) / n
    sel = [None, None, None]
    sel[2 - axis] = slice(None)
    L = (pos < 0.5)[tuple(sel)]
    q = 1.0 / math.sqrt(4.0 * math.pi)
    left_v, right_v = (1.2, 0.01, 0.5), (0.0, 0.0, 0.0)
    left_b, right_b = (2.0 * q, 3.6 * q, 2.0 * q), (2.0 * q, 4.0 * q, 2.0 * q)
    vel = [None] * 3
    bfield = [None] * 3
    for k in range(3):
        a = (axis + k) % 3
        vel[a] = np.broadcast_to(np.where(L, left_v[k], right_v[k]), shape).astype(np.float64)
        bfield[a] = np.broadcast_to(np.where(L, left_b[k], right_b[k]), shape).astype(np.float64)
    rho = np.where(L, 1.08, 1.0)
    p = np.where(L, 0.95, 1.0)
    return assemble(rho, tuple(vel), p, tuple(bfield), tuple(bfield), gamma, shape)


def blast2d(n: int, gamma: float = 5.0 / 3.0):
    """2D blast wave of Sec. 5.2.2 on n x n: rho 1, v 0, B = (1, 1, 0) / sqrt2,
    p 10 inside r < 0.1 about (0.5, 0.5), 0.1 outside (the second pressure
    printed with the other constants is taken as a stray)."""
    return blast(n, nz=1, gamma=gamma)


ROTORS = {1: {"v0": 2.0, "p": 1.0, "gamma": 1.4, "bx": 5.0, "t_max": 0.15},
          2: {"v0": 1.0, "p": 0.5, "gamma": 5.0 / 3.0, "bx": 2.5, "t_max": 0.295}}


def rotor(n: int, which: int = 1):
    """MHD rotor of Sec. 5.2.3 on n x n: dense disk (rho 10) of radius 0.1
    spinning rigidly with speed v0 at its edge, a taper to the ambient rho 1
    at rest between r 0.1 and 0.115 with f = (0.115 - r) / 0.015,
    rho = 1 + 9 f and v = f v0 (-(y - 0.5), (x - 0.5)) / r (the taper's v_y
    sign is read as that of the disk, which keeps v continuous at r = 0.1),
    uniform p and B = (bx / sqrt(4 pi), 0, 0). Parameter set `which` = 1 or 2."""
    c = ROTORS[which]
    shape = (1, n, n)
    x, y, _ = _grid(n, n, 1, "ccc")
    dx, dy = x - 0.5, y - 0.5
    r = np.sqrt(dx * dx + dy * dy) + 0.0 * (x + y)
    r0, r1 = 0.1, 0.115
    f = (r1 - r) / (r1 - r0)
    inside, taper = r < r0, (r >= r0) & (r < r1)
    rho = np.where(inside, 10.0, np.where(taper, 1.0 + 9.0 * f, 1.0))
    rs = np.where(r > 0.0, r, 1.0)
    vx = np.where(inside, -c["v0"] * dy / r0, np.where(taper, -f * c["v0"] * dy / rs, 0.0))
    vy = np.where(inside, c["v0"] * dx / r0, np.where(taper, f * c["v0"] * dx / rs, 0.0))
    b = (np.full(shape, c["bx"] / math.sqrt(4.0 * math.pi)), np.zeros(shape), np.zeros(shape))
    return assemble(rho, (vx, vy, 0.0), c["p"], b, b, c["gamma"], shape)


# --------------------------------------------------------------------------
# Smooth states with known behaviour
# --------------------------------------------------------------------------

def uniform(nx, ny, nz, rho=1.0, vel=(0.0, 0.0, 0.0), p=1.0, bvec=(0.0, 0.0, 0.0), gamma=5.0 / 3.0):
    shape = (nz, ny, nx)
    b = tuple(np.full(shape, float(c)) for c in bvec)
    return assemble(rho, vel, p, b, b, gamma, shape)


def wavevector(nx, ny, nz, kvec):
    """Physical wave vector of integer mode numbers kvec on the box."""
    h = cell_width(nx, ny, nz)
    side = np.array([nx * h, ny * h, nz * h])
    return 2.0 * math.pi * np.asarray(kvec, dtype=np.float64) / side


def linear_wave(nx, ny, nz, kvec, rho0, p0, vel0, bvec0, gamma, drho=0.0, dv=(0.0, 0.0, 0.0), dp=0.0,
                db=0.0, db_dir=(0.0, 0.0, 0.0), phase=0.0):
    """Plane wave on a uniform background: every perturbation varies as
    sin(theta), theta = k . x - phase with k_a = 2 pi kvec_a / L_a (kvec
    integer per axis, L_a the box side) so the pattern is periodic.

    The field perturbation db * db_dir (db_dir a unit vector orthogonal to kvec)
    is the discrete curl of a = db/|k| (k_hat x db_dir) cos(theta) on the edges,
    so it is divergence free to round-off."""
    shape = (nz, ny, nx)
    k = wavevector(nx, ny, nz, kvec)
    kn = float(np.linalg.norm(k))
    ndir = np.asarray(db_dir, dtype=np.float64)

    def theta(x, y, z):
        return k[0] * x + k[1] * y + k[2] * z - phase

    xc, yc, zc = _grid(nx, ny, nz, "ccc")
    th = theta(xc, yc, zc)
    sn = np.sin(th)
    rho = rho0 + drho * sn
    vel = tuple(vel0[a] + dv[a] * sn for a in range(3))
    p = p0 + dp * sn
    if db != 0.0:
        w = np.cross(k / kn, ndir) * (db / kn)

        def comp(a):
            return lambda x, y, z: w[a] * np.cos(theta(x, y, z))

        bx, by, bz = curl_faces(comp(0), comp(1), comp(2), nx, ny, nz)
        bface = (bx + bvec0[0], by + bvec0[1], bz + bvec0[2])
    else:
        bface = tuple(np.full(shape, float(bvec0[a])) for a in range(3))
    bcen = tuple(bvec0[a] + db * ndir[a] * sn for a in range(3))
    return assemble(rho, vel, p, bface, bcen, gamma, shape)


def random_smooth(nx, ny, nz, seed, gamma=5.0 / 3.0, amp=0.2, modes=3, bmean=(0.6, -0.3, 0.4), vmean=(0.1, -0.2, 0.15)):
    """Smooth periodic state with random low Fourier modes (seeded, NumPy PCG64):
    positive density and pressure, non-zero velocity, and a field made of a
    uniform part plus the discrete curl of a random periodic potential."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nz, ny, nx)
    xc, yc, zc = _grid(nx, ny, nz, "ccc")
    h = cell_width(nx, ny, nz)
    side = (nx * h, ny * h, nz * h)

    def kphys(kx, ky, kz):
        return (2 * math.pi * kx / side[0], 2 * math.pi * ky / side[1], 2 * math.pi * kz / side[2])

    def field(x, y, z, coef):
        out = 0.0
        for (kx, ky, kz, a, ph) in coef:
            k = kphys(kx, ky, kz)
            out = out + a * np.sin(k[0] * x + k[1] * y + k[2] * z + ph)
        return out

    # at most one period per four cells along each axis (uniform along axes of < 4 cells)
    kmax = [min(modes, n // 4) for n in (nx, ny, nz)]

    def draw():
        return [(int(rng.integers(0, kmax[0] + 1)), int(rng.integers(0, kmax[1] + 1)),
                 int(rng.integers(0, kmax[2] + 1)),
                 float(rng.uniform(-1, 1)), float(rng.uniform(0, 2 * math.pi))) for _ in range(4)]

    rho = 1.0 + amp * field(xc, yc, zc, draw())
    p = 1.0 + amp * field(xc, yc, zc, draw())
    vel = tuple(vmean[a] + amp * field(xc, yc, zc, draw()) for a in range(3))
    acoef = [draw() for _ in range(3)]
    scale = amp / (2 * math.pi * max(modes, 1))
    pot = [lambda x, y, z, c=acoef[a]: scale * field(x, y, z, c) for a in range(3)]
    bx, by, bz = curl_faces(pot[0], pot[1], pot[2], nx, ny, nz)
    bface = (bx + bmean[0], by + bmean[1], bz + bmean[2])

    # analytic centred field: curl of the continuous potential at cell centres
    def dfield(x, y, z, coef, axis):
        out = 0.0
        for (kx, ky, kz, a, ph) in coef:
            k = kphys(kx, ky, kz)
            out = out + a * k[axis] * np.cos(k[0] * x + k[1] * y + k[2] * z + ph)
        return out

    def d(a, axis):
        return scale * dfield(xc, yc, zc, acoef[a], axis)

    bcx = bmean[0] + d(2, 1) - d(1, 2)
    bcy = bmean[1] + d(0, 2) - d(2, 0)
    bcz = bmean[2] + d(1, 0) - d(0, 1)
    return assemble(rho, vel, p, bface, (bcx, bcy, bcz), gamma, shape)


# --------------------------------------------------------------------------
# Batched workload: many periodic linear Alfven waves of uneven sizes
# --------------------------------------------------------------------------

BATCH_SIZES = (32, 48, 64, 96, 128)


def alfven_batch_specs(count: int, seed: int = MASTER_SEED + 400, sizes=BATCH_SIZES, gamma: float = 5.0 / 3.0):
    """Seeded parameters of `count` Alfven-wave problems: cubic grid n drawn
    uniformly from `sizes`, unit background field along a uniformly random
    direction b (redrawn while |k.b| < 0.1 or |k x b| < 0.1 for the wave
    normal k = (1,1,1)/sqrt3, so the wave neither stalls nor degenerates) and
    amplitude uniform in [1e-4, 1e-2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    khat = np.ones(3) / math.sqrt(3.0)
    specs = []
    for _ in range(count):
        n = int(rng.choice(np.asarray(sizes)))
        while True:
            b = rng.normal(size=3)
            b /= np.linalg.norm(b)
            if abs(float(khat @ b)) >= 0.1 and np.linalg.norm(np.cross(khat, b)) >= 0.1:
                break
        amp = float(rng.uniform(1e-4, 1e-2))
        specs.append({"n": n, "b0": tuple(float(c) for c in b), "amp": amp, "gamma": gamma})
    return specs


def alfven_111(n: int, b0, amp: float, gamma: float = 5.0 / 3.0, rho0: float = 1.0, dtype=np.float64):
    """Linear Alfven wave with wave vector 2 pi (1,1,1) on a periodic n^3 unit
    box: rho = rho0, p = 1/gamma, background field b0, field perturbation amp
    along n = k x b0 (unit), velocity -sign(k.b0) amp n / sqrt(rho0); the face
    field is the discrete curl of the edge potential (k x n) amp / |k| cos(k.x).

    Every quantity depends on the cell position only through m = i + j + k, so
    it is tabulated over m (3n - 2 values) and gathered; this is the same state
    linear_wave builds, without evaluating sin/cos at every cell."""
    b0 = np.asarray(b0, dtype=np.float64)
    khat = np.ones(3) / math.sqrt(3.0)
    ndir = np.cross(khat, b0)
    ndir /= np.linalg.norm(ndir)
    sgn = 1.0 if float(khat @ b0) >= 0.0 else -1.0
    h = 1.0 / n
    kn = 2.0 * math.pi * math.sqrt(3.0)
    w = np.cross(khat, ndir) * (amp / kn)
    m = np.arange(3 * n - 2, dtype=np.float64)
    sn = np.sin(2.0 * math.pi * h * (m + 1.5))                                    # cell centres
    dc = (np.cos(2.0 * math.pi * h * (m + 1.5)) - np.cos(2.0 * math.pi * h * (m + 0.5))) / h   # edge differences
    idx = (np.arange(n)[None, None, :] + np.arange(n)[None, :, None] + np.arange(n)[:, None, None])
    p0 = 1.0 / gamma
    s = np.empty((8, n, n, n), dtype=dtype)
    dv = -sgn * amp / math.sqrt(rho0) * ndir
    bc = [b0[a] + amp * ndir[a] * sn for a in range(3)]
    mom = [rho0 * dv[a] * sn for a in range(3)]
    kin = 0.5 * rho0 * ((dv[0] * sn) ** 2 + (dv[1] * sn) ** 2 + (dv[2] * sn) ** 2)
    mag = 0.5 * (bc[0] ** 2 + bc[1] ** 2 + bc[2] ** 2)
    s[0] = rho0
    for a in range(3):
        s[1 + a] = np.take(mom[a], idx)
    s[4] = np.take(p0 / (gamma - 1.0) + kin + mag, idx)
    curl = (w[2] - w[1], w[0] - w[2], w[1] - w[0])
    for a in range(3):
        s[5 + a] = np.take(b0[a] + curl[a] * dc, idx)
    return s


# --------------------------------------------------------------------------
# Serving workload: blast waves and extruded Orszag-Tang vortices
# --------------------------------------------------------------------------

SERVE_SIZES = (32, 64, 96, 128, 160, 192)


def serving_specs(count: int, seed: int = MASTER_SEED + 500, sizes=SERVE_SIZES, nsteps: int = 100):
    """Seeded request parameters: half 3D blast waves (ambient p 0.1, p_in
    uniform in [1, 100], radius uniform in [0.05, 0.15], uniform field of
    magnitude uniform in [0, 1] along a uniformly random direction), half
    Orszag-Tang vortices extruded along z; cubic grid n drawn from `sizes`;
    FP32 or FP64 with equal probability; `nsteps` full steps each."""
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for _ in range(count):
        kind = "blast" if rng.uniform() < 0.5 else "vortex"
        n = int(rng.choice(np.asarray(sizes)))
        dtype = 1 if rng.uniform() < 0.5 else 0
        sp = {"kind": kind, "n": n, "dtype": dtype, "nsteps": nsteps, "gamma": 5.0 / 3.0}
        if kind == "blast":
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            bmag = float(rng.uniform(0.0, 1.0))
            sp.update(p_in=float(rng.uniform(1.0, 100.0)), radius=float(rng.uniform(0.05, 0.15)),
                      bvec=tuple(float(c) for c in bmag * d))
        specs.append(sp)
    return specs


def serving_state(sp: dict, dtype=np.float64):
    """Initial state of one serving request, written straight into an array of
    `dtype`: the same values as blast(n, p_in, 0.1, radius, bvec) or
    orszag_tang(n, nz=n), built from 1D / 2D factors instead of full-size
    temporaries."""
    n, gamma = sp["n"], sp["gamma"]
    h = 1.0 / n
    s = np.empty((8, n, n, n), dtype=dtype)
    c = (np.arange(n) + 0.5) * h
    if sp["kind"] == "blast":
        bv = sp["bvec"]
        mag = 0.5 * (bv[0] ** 2 + bv[1] ** 2 + bv[2] ** 2)
        e_in = sp["p_in"] / (gamma - 1.0) + 0.0 + mag
        e_out = 0.1 / (gamma - 1.0) + 0.0 + mag
        d2 = (c - 0.5) ** 2
        r2 = (d2[None, None, :] + d2[None, :, None]) + d2[:, None, None]
        s[0] = 1.0
        s[1:4] = 0.0
        s[4] = np.where(r2 < sp["radius"] ** 2, e_in, e_out)
        for a in range(3):
            s[5 + a] = bv[a]
        return s
    b0 = 1.0 / math.sqrt(4.0 * math.pi)
    rho = 25.0 / (36.0 * math.pi)
    p = 5.0 / (12.0 * math.pi)
    vx = -np.sin(2 * math.pi * c)[:, None] + 0.0 * c[None, :]    # (y, x)
    vy = np.sin(2 * math.pi * c)[None, :] + 0.0 * c[:, None]
    bx = -b0 * np.sin(2 * math.pi * c)[:, None] + 0.0 * c[None, :]
    by = b0 * np.sin(4 * math.pi * c)[None, :] + 0.0 * c[:, None]
    kin = 0.5 * rho * (vx ** 2 + vy ** 2 + 0.0 ** 2)
    mag = 0.5 * (bx ** 2 + by ** 2 + 0.0 ** 2)
    s[0] = rho
    s[1] = (rho * vx)[None]
    s[2] = (rho * vy)[None]
    s[3] = 0.0
    s[4] = (p / (gamma - 1.0) + kin + mag)[None]
    s[5] = bx[None]
    s[6] = by[None]
    s[7] = 0.0
    return s

"""Shared test helpers: state symmetries, linear-wave setups, an exact Euler
Riemann solver (textbook), and error norms. No solver arithmetic lives here."""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq

from paper_0908_4362_amd import problems as P

GAMMA53 = 5.0 / 3.0


# ---------------------------------------------------------------- symmetries

def rotate_state(s: np.ndarray) -> np.ndarray:
    """Cyclic relabelling of axes x->y, y->z, z->x of a state (8, nz, ny, nx).

    Cell (i, j, k) moves to (k, i, j); vector components follow their axis."""
    out = np.empty((8,) + (s.shape[2], s.shape[3], s.shape[1]), dtype=s.dtype)
    # new array index order (z', y', x') = (y, x, z): new x' = old z, y' = old x, z' = old y
    def mv(a):
        return np.ascontiguousarray(np.transpose(a, (1, 2, 0)))
    out[0] = mv(s[0])
    out[4] = mv(s[4])
    for a in range(3):
        out[1 + (a + 1) % 3] = mv(s[1 + a])
        out[5 + (a + 1) % 3] = mv(s[5 + a])
    return out


def mirror_x(s: np.ndarray) -> np.ndarray:
    """Reflection x -> 1 - x of a state whose B_x is uniform along x (so the
    face re-indexing does not matter): cells i -> n-1-i, m_x -> -m_x,
    B_x -> -B_x (B -> -B maps solutions to solutions)."""
    out = s[..., ::-1].copy()
    out[1] = -out[1]
    out[5] = -out[5]
    return out


def point_reflect_xy(s: np.ndarray) -> np.ndarray:
    """(x, y) -> (1 - x, 1 - y) of a 2D periodic state, i.e. a rotation by pi
    about z: cells (i, j) -> (n-1-i, n-1-j); x-faces i -> (n - i) mod n; the x
    and y components of vectors change sign, the z components do not."""
    out = np.empty_like(s)
    cell = s[..., ::-1, ::-1]
    for f in (0, 3, 4, 7):
        out[f] = cell[f]
    for f in (1, 2):
        out[f] = -cell[f]
    bx = s[5][..., ::-1, :]            # y is a cell index for B_x
    out[5] = -np.roll(bx[..., ::-1], 1, axis=-1)
    by = s[6][..., :, ::-1]            # x is a cell index for B_y
    out[6] = -np.roll(by[..., ::-1, :], 1, axis=-2)
    return out


def symmetrize(s, op):
    """(s + op(s)) / 2, exactly invariant under an involution op that only
    permutes entries and flips signs."""
    return 0.5 * (s + op(s))


# ---------------------------------------------------------------- norms

def rel_linf(a, b):
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def rel_l1(a, b):
    den = np.sum(np.abs(b))
    return float(np.sum(np.abs(a - b)) / (den if den > 0 else 1.0))


# ---------------------------------------------------------------- waves

def wave_setup(kind, nx, ny, nz, kvec, amp, b0dir=(1.0, 0.6, 0.3), gamma=GAMMA53, rho0=1.0, p0=1.0,
               vflow=(0.0, 0.0, 0.0)):
    """Closed-form linear MHD plane waves on a uniform background moving with
    vflow. Returns (make(phase), omega) where make builds the state at a given
    phase and omega = |k| * phase speed (intrinsic speed plus flow along k).

    The freezing speed |v_n| + c_f has a kink where the normal velocity changes
    sign; waves on a background at rest whose velocity perturbation is along k
    therefore converge at a reduced rate, so compressive waves are run on a
    background flow along k."""
    k = P.wavevector(nx, ny, nz, kvec)
    kn = float(np.linalg.norm(k))
    kh = k / kn
    cs2 = gamma * p0 / rho0
    if kind == "alfven":
        B0 = np.asarray(b0dir, dtype=float)
        B0 = B0 / np.linalg.norm(B0)
        n = np.cross(kh, B0)
        n = n / np.linalg.norm(n)
        sgn = math.copysign(1.0, float(B0 @ kh))
        speed = abs(float(B0 @ kh)) / math.sqrt(rho0)

        def make(ph):
            return P.linear_wave(nx, ny, nz, kvec, rho0, p0, vflow, tuple(B0), gamma,
                                 dv=tuple(-sgn * amp * n / math.sqrt(rho0)), db=amp, db_dir=tuple(n), phase=ph)
    elif kind == "sound":
        speed = math.sqrt(cs2)

        def make(ph):
            return P.linear_wave(nx, ny, nz, kvec, rho0, p0, vflow, (0.0, 0.0, 0.0), gamma, drho=amp,
                                 dv=tuple(speed * amp / rho0 * kh), dp=cs2 * amp, phase=ph)
    elif kind == "fast_perp":
        # field orthogonal to k: fast speed sqrt(cs^2 + vA^2), dB = B0 drho / rho0
        B0 = np.asarray(b0dir, dtype=float)
        B0 = B0 - (B0 @ kh) * kh
        B0 = B0 / np.linalg.norm(B0)
        speed = math.sqrt(cs2 + 1.0 / rho0)

        def make(ph):
            return P.linear_wave(nx, ny, nz, kvec, rho0, p0, vflow, tuple(B0), gamma, drho=amp,
                                 dv=tuple(speed * amp / rho0 * kh), dp=cs2 * amp, db=amp / rho0,
                                 db_dir=tuple(B0), phase=ph)
    elif kind in ("fast", "slow"):
        # oblique magnetosonic waves: B0 = B_par k_hat + B_perp t_hat (|B0| = 1);
        # speeds from (s^2 - cs^2)(s^2 - vAx^2) = vAy^2 s^2 with vAx, vAy the
        # Alfven speeds of B_par, B_perp; eigenvector for drho = amp
        B0 = np.asarray(b0dir, dtype=float)
        B0 = B0 / np.linalg.norm(B0)
        bpar = float(B0 @ kh)
        bper = B0 - bpar * kh
        by = float(np.linalg.norm(bper))
        t = bper / by
        vax2, vay2 = bpar ** 2 / rho0, by ** 2 / rho0
        a = cs2 + vax2 + vay2
        root = math.sqrt(a * a - 4 * cs2 * vax2)
        speed = math.sqrt(0.5 * (a + root) if kind == "fast" else 0.5 * (a - root))
        dvk = speed * amp / rho0
        dbt = by * speed * dvk / (speed ** 2 - vax2)
        dvt = -bpar * dbt / (speed * rho0)

        def make(ph):
            return P.linear_wave(nx, ny, nz, kvec, rho0, p0, vflow, tuple(B0), gamma, drho=amp,
                                 dv=tuple(dvk * kh + dvt * t), dp=cs2 * amp, db=dbt, db_dir=tuple(t), phase=ph)
    elif kind == "entropy":
        # density wave carried by a uniform flow vflow at uniform pressure
        B0 = np.asarray(b0dir, dtype=float)
        speed = 0.0

        def make(ph):
            return P.linear_wave(nx, ny, nz, kvec, rho0, p0, vflow, tuple(B0), gamma, drho=amp, phase=ph)
    else:
        raise ValueError(kind)
    # a uniform background flow carries every mode (Galilean shift)
    return make, kn * (speed + float(np.asarray(vflow) @ kh))


# ---------------------------------------------------------------- exact Riemann (Euler)

def exact_riemann(left, right, gamma, xi):
    """Exact solution of the 1D Euler Riemann problem (Toro, ch. 4) sampled at
    xi = (x - x0) / t. left/right = (rho, u, p). Returns rho, u, p arrays."""
    rL, uL, pL = left
    rR, uR, pR = right
    cL, cR = math.sqrt(gamma * pL / rL), math.sqrt(gamma * pR / rR)
    g1 = (gamma - 1) / (2 * gamma)

    def fk(p, rk, pk, ck):
        if p > pk:
            A = 2 / ((gamma + 1) * rk)
            B = (gamma - 1) / (gamma + 1) * pk
            return (p - pk) * math.sqrt(A / (p + B))
        return 2 * ck / (gamma - 1) * ((p / pk) ** g1 - 1)

    fn = lambda p: fk(p, rL, pL, cL) + fk(p, rR, pR, cR) + (uR - uL)
    ps = brentq(fn, 1e-12, 100 * max(pL, pR), xtol=1e-15, rtol=1e-15)
    us = 0.5 * (uL + uR) + 0.5 * (fk(ps, rR, pR, cR) - fk(ps, rL, pL, cL))
    out = np.zeros((3, len(xi)))
    gr = (gamma - 1) / (gamma + 1)
    for n, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pL:
                SL = uL - cL * math.sqrt((gamma + 1) / (2 * gamma) * ps / pL + g1)
                if s <= SL:
                    out[:, n] = (rL, uL, pL)
                else:
                    rs = rL * ((ps / pL + gr) / (gr * ps / pL + 1))
                    out[:, n] = (rs, us, ps)
            else:
                cs = cL * (ps / pL) ** g1
                SH, ST = uL - cL, us - cs
                if s <= SH:
                    out[:, n] = (rL, uL, pL)
                elif s >= ST:
                    out[:, n] = (rL * (ps / pL) ** (1 / gamma), us, ps)
                else:
                    u = 2 / (gamma + 1) * (cL + (gamma - 1) / 2 * uL + s)
                    c = 2 / (gamma + 1) * (cL + (gamma - 1) / 2 * (uL - s))
                    rho = rL * (c / cL) ** (2 / (gamma - 1))
                    out[:, n] = (rho, u, pL * (c / cL) ** (1 / g1))
        else:
            if ps > pR:
                SR = uR + cR * math.sqrt((gamma + 1) / (2 * gamma) * ps / pR + g1)
                if s >= SR:
                    out[:, n] = (rR, uR, pR)
                else:
                    rs = rR * ((ps / pR + gr) / (gr * ps / pR + 1))
                    out[:, n] = (rs, us, ps)
            else:
                cs = cR * (ps / pR) ** g1
                SH, ST = uR + cR, us + cs
                if s >= SH:
                    out[:, n] = (rR, uR, pR)
                elif s <= ST:
                    out[:, n] = (rR * (ps / pR) ** (1 / gamma), us, ps)
                else:
                    u = 2 / (gamma + 1) * (-cR + (gamma - 1) / 2 * uR + s)
                    c = 2 / (gamma + 1) * (cR - (gamma - 1) / 2 * (uR - s))
                    rho = rR * (c / cR) ** (2 / (gamma - 1))
                    out[:, n] = (rho, u, pR * (c / cR) ** (1 / g1))
    return out

"""CPU oracle for the relaxing-TVD + constrained-transport MHD step.

TEST INFRASTRUCTURE ONLY. This is the slow, serial, FP64 reference the GPU
library is checked against (plain C in ``mhd_oracle.c``, loaded here through
ctypes; ``set_threads(n)`` switches to the OpenMP build of the same source,
which shares the pencils of each sweep among n threads and gives the same
bits). Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it; the GPU library never does.

States are numpy float64 arrays of shape (8, nz, ny, nx): fields rho, m_x,
m_y, m_z, E, B_x, B_y, B_z, x fastest; B_d holds the value on the lower
d-face of each cell (Sec. 3, eq. equat_b).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mhd_oracle.c")
_SO = os.path.join(_HERE, "liborc_mhd.so")
_SO_OMP = os.path.join(_HERE, "liborc_mhd_omp.so")
_libs = {}
_threads = 1

PERIODIC, OUTFLOW = 0, 1

# -O3 without FMA contraction or fast-math: every expression rounds as written
_CFLAGS = ["-O3", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def _compile(out, extra):
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *_CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, out)


def build(force: bool = False) -> str:
    """Compile the oracle: the serial library and the OpenMP one (the same
    source with its pencil loops shared among threads, same bits)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "mhd_oracle.h")))
    for so, extra in ((_SO, []), (_SO_OMP, ["-fopenmp"])):
        if force or not os.path.exists(so) or os.path.getmtime(so) < newest:
            _compile(so, extra)
    return _SO


def set_threads(n: int) -> int:
    """Run the oracle on n threads (1: the serial build; more: the OpenMP
    build with n threads). Returns the thread count in use."""
    global _threads
    _threads = max(1, int(n))
    lib = _load()
    return int(lib.orc_set_threads(_threads)) if _threads > 1 else 1


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("gamma", ctypes.c_double), ("bc", ctypes.c_int)]


def _load():
    key = "omp" if _threads > 1 else "serial"
    lib = _libs.get(key)
    if lib is None:
        build()
        lib = ctypes.CDLL(_SO_OMP if key == "omp" else _SO)
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(_Grid)
        lib.orc_vanleer.restype = ctypes.c_double
        lib.orc_vanleer.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_flux_speed.restype = None
        lib.orc_flux_speed.argtypes = [dp, dp, ctypes.c_double, dp, dp]
        for name in ("orc_fluid_sweep", "orc_ct_sweep"):
            fn = getattr(lib, name)
            fn.restype = None
            fn.argtypes = [gp, dp, dp, ctypes.c_int, ctypes.c_double]
        lib.orc_cmax.restype = ctypes.c_double
        lib.orc_cmax.argtypes = [gp, dp]
        lib.orc_dt.restype = ctypes.c_int
        lib.orc_dt.argtypes = [ctypes.c_double] * 4 + [dp, dp]
        lib.orc_step_dt.restype = None
        lib.orc_step_dt.argtypes = [gp, dp, ctypes.c_double, ctypes.c_longlong]
        lib.orc_step.restype = ctypes.c_int
        lib.orc_step.argtypes = [gp, dp, ctypes.c_double, ctypes.c_double, dp,
                                 ctypes.POINTER(ctypes.c_longlong)]
        lib.orc_divb_max.restype = ctypes.c_double
        lib.orc_divb_max.argtypes = [gp, dp]
        lib.orc_set_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _libs[key] = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Grid:
    """Grid sizes, adiabatic index and boundary condition (0 periodic, 1 outflow)."""

    def __init__(self, nx: int, ny: int, nz: int, gamma: float, bc: int = PERIODIC):
        self.n = (int(nx), int(ny), int(nz))
        self.gamma = float(gamma)
        self.bc = int(bc)
        self._c = _Grid((ctypes.c_int * 3)(*self.n), self.gamma, self.bc)

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (8, nz, ny, nx)


def _as_state(g: Grid, s) -> np.ndarray:
    a = np.ascontiguousarray(s, dtype=np.float64)
    if a.shape != g.shape:
        a = a.reshape(g.shape)
    return a


def vanleer(a: float, b: float) -> float:
    return _load().orc_vanleer(a, b)


def flux_speed(u, b, gamma: float):
    """Flux (rotated, normal components first) and freezing speed of one cell."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    F = np.zeros(5)
    c = np.zeros(1)
    _load().orc_flux_speed(_ptr(u), _ptr(b), gamma, _ptr(F), _ptr(c))
    return F, float(c[0])


def fluid_sweep(g: Grid, s, d: int, dt: float) -> np.ndarray:
    a = _as_state(g, s)
    out = np.empty_like(a)
    _load().orc_fluid_sweep(ctypes.byref(g._c), _ptr(a), _ptr(out), d, dt)
    return out


def ct_sweep(g: Grid, s, d: int, dt: float) -> np.ndarray:
    a = _as_state(g, s)
    out = np.empty_like(a)
    _load().orc_ct_sweep(ctypes.byref(g._c), _ptr(a), _ptr(out), d, dt)
    return out


def cmax(g: Grid, s) -> float:
    return _load().orc_cmax(ctypes.byref(g._c), _ptr(_as_state(g, s)))


def dt_rule(cmax_value: float, cfl: float, t: float, t_stop: float | None):
    dt = np.zeros(1)
    tn = np.zeros(1)
    rc = _load().orc_dt(cmax_value, cfl, t, -1.0 if t_stop is None else t_stop, _ptr(dt), _ptr(tn))
    if rc:
        raise FloatingPointError("non-finite or non-positive c_max")
    return float(dt[0]), float(tn[0])


def step_dt(g: Grid, s, dt: float, step: int) -> np.ndarray:
    a = _as_state(g, s).copy()
    _load().orc_step_dt(ctypes.byref(g._c), _ptr(a), dt, step)
    return a


def run(g: Grid, s, nsteps: int, cfl: float, t: float = 0.0, step: int = 0, t_stop: float | None = None):
    """Advance nsteps full steps; returns (state, t, step)."""
    a = _as_state(g, s).copy()
    tt = np.array([t], dtype=np.float64)
    ss = ctypes.c_longlong(step)
    lib = _load()
    for _ in range(nsteps):
        rc = lib.orc_step(ctypes.byref(g._c), _ptr(a), cfl, -1.0 if t_stop is None else t_stop, _ptr(tt),
                          ctypes.byref(ss))
        if rc:
            raise FloatingPointError("non-finite or non-positive c_max")
    return a, float(tt[0]), int(ss.value)


def divb_max(g: Grid, s) -> float:
    return _load().orc_divb_max(ctypes.byref(g._c), _ptr(_as_state(g, s)))

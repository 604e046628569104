"""Thin ctypes binding of the C ABI in include/mhd.h, include/mhd_batch.h and
include/mhd_server.h (same names).

Only argument marshalling lives here: every step of the computation runs in
the HIP library. Host states are numpy arrays of shape (8, nz, ny, nx) (or any
contiguous buffer of 8*nx*ny*nz elements of the handle's dtype); device
states are torch tensors on the GPU (or raw device addresses).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhd.so")

MHD_OK, MHD_ERR_ARG, MHD_ERR_OOM, MHD_ERR_DEVICE, MHD_ERR_NONFINITE = 0, -1, -2, -3, -4
MHD_BC_PERIODIC, MHD_BC_OUTFLOW = 0, 1
MHD_F32, MHD_F64 = 0, 1
(MHD_K_CFL, MHD_K_FLUID_X, MHD_K_FLUID_Y, MHD_K_FLUID_Z, MHD_K_CT_X, MHD_K_CT_Y, MHD_K_CT_Z, MHD_K_CTFLUID_X,
 MHD_K_CTFLUID_Y, MHD_K_CTFLUID_Z, MHD_K_COUNT) = range(11)
KERNEL_KINDS = ("cfl", "fluid_x", "fluid_y", "fluid_z", "ct_x", "ct_y", "ct_z", "ctfluid_x", "ctfluid_y", "ctfluid_z")
MHD_D_PRESSURE, MHD_D_MAGNETIC_PRESSURE, MHD_D_SPEED, MHD_D_DIVB, MHD_D_CFL_SPEED, MHD_D_COUNT = range(6)

_lib = None


class MHDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("mhd error %d: %s" % (code, msg))
        self.code = code


def lib():
    """Load libmhd.so; fail loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmhd.so is not built; run `python -m paper_0908_4362_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        sig = {
            "mhd_create": ([i, i, i, d, i, i, ctypes.POINTER(vp)], i),
            "mhd_destroy": ([vp], i),
            "mhd_set_stream": ([vp, vp], i),
            "mhd_set_graphs": ([vp, i], i),
            "mhd_set_fusion": ([vp, i], i),
            "mhd_set_state": ([vp, vp], i),
            "mhd_set_state_device": ([vp, vp], i),
            "mhd_get_state": ([vp, vp], i),
            "mhd_get_state_device": ([vp, vp], i),
            "mhd_step": ([vp, i, d], i),
            "mhd_divb_max": ([vp, ctypes.POINTER(d)], i),
            "mhd_divb_max_noalloc": ([vp, i, i, i, i, i, vp, vp], i),
            "mhd_get_time": ([vp, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_int64)], i),
            "mhd_set_time": ([vp, d, ctypes.c_int64], i),
            "mhd_set_stop_time": ([vp, d], i),
            "mhd_last_error": ([], ctypes.c_char_p),
            "mhd_fluid_sweep": ([vp, i, d], i),
            "mhd_ct_sweep": ([vp, i, d], i),
            "mhd_cmax": ([vp, ctypes.POINTER(d)], i),
            "mhd_step_dt": ([vp, d, ctypes.c_int64], i),
            "mhd_state_bytes": ([i, i, i, i], ctypes.c_size_t),
            "mhd_workspace_bytes": ([i, i, i, i], ctypes.c_size_t),
            "mhd_bind_workspace": ([vp, vp, ctypes.c_size_t], i),
            "mhd_timing": ([vp, i], i),
            "mhd_timing_read": ([vp, i, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_int64)], i),
            "mhd_diagnostic": ([vp, i, i, i, vp], i),
            "mhd_batch_create": ([i, ctypes.POINTER(vp)], i),
            "mhd_batch_destroy": ([vp], i),
            "mhd_batch_set_stream": ([vp, vp], i),
            "mhd_batch_problem_bytes": ([i, i, i, i], ctypes.c_size_t),
            "mhd_batch_add": ([vp, i, i, i, d, i, vp, ctypes.POINTER(i)], i),
            "mhd_batch_add_device": ([vp, i, i, i, d, i, vp, ctypes.POINTER(i)], i),
            "mhd_batch_remove": ([vp, i], i),
            "mhd_batch_count": ([vp, ctypes.POINTER(i), ctypes.POINTER(ctypes.c_size_t)], i),
            "mhd_batch_step": ([vp, i, d], i),
            "mhd_batch_get_state": ([vp, i, vp], i),
            "mhd_batch_get_state_device": ([vp, i, vp], i),
            "mhd_batch_get_time": ([vp, i, ctypes.POINTER(d), ctypes.POINTER(ctypes.c_int64)], i),
            "mhd_batch_set_stop_time": ([vp, i, d], i),
            "mhd_batch_status": ([vp, i], i),
            "mhd_batch_set_graphs": ([vp, i], i),
            "mhd_batch_autotune": ([vp, i], i),
            "mhd_batch_tile": ([vp, i, i, ctypes.POINTER(i), ctypes.POINTER(i)], i),
            "mhd_batch_set_tile": ([vp, i, i, i, i], i),
            "mhd_batch_problem_layout": ([i, i, i, i, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                          ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)], i),
            "mhd_batch_add_inplace": ([vp, i, i, i, d, i, vp, vp, ctypes.POINTER(i)], i),
            "mhd_batch_record": ([vp, vp], i),
            "mhd_server_now": ([], d),
            "mhd_server_create": ([ctypes.c_size_t, d, ctypes.POINTER(vp)], i),
            "mhd_server_destroy": ([vp], i),
            "mhd_server_set_max_cells": ([vp, ctypes.c_int64], i),
            "mhd_server_submit": ([vp, i, i, i, d, i, i, vp, i, ctypes.POINTER(i)], i),
            "mhd_server_submit_ref": ([vp, i, i, i, d, i, i, vp, i, ctypes.POINTER(i)], i),
            "mhd_server_tick": ([vp, ctypes.POINTER(i), ctypes.POINTER(i)], i),
            "mhd_server_poll": ([vp, ctypes.POINTER(i)], i),
            "mhd_server_info": ([vp, i, ctypes.POINTER(i), ctypes.POINTER(d), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(i), ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d)], i),
            "mhd_server_take": ([vp, i, vp], i),
            "mhd_server_stats": ([vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int64)], i),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def mhd_last_error() -> str:
    return lib().mhd_last_error().decode()


def _check(rc: int):
    if rc != MHD_OK:
        raise MHDError(rc, mhd_last_error())


def _np_dtype(dtype: int):
    return np.float64 if dtype == MHD_F64 else np.float32


def _dev_ptr(x) -> int:
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def mhd_create(nx: int, ny: int, nz: int, gamma: float, bc: int, dtype: int):
    h = ctypes.c_void_p()
    _check(lib().mhd_create(nx, ny, nz, gamma, bc, dtype, ctypes.byref(h)))
    return h


def mhd_destroy(h):
    _check(lib().mhd_destroy(h))


def mhd_set_stream(h, stream):
    """stream: a torch.cuda.Stream, a raw hipStream_t address, or None."""
    ptr = None if stream is None else (stream if isinstance(stream, int) else int(stream.cuda_stream))
    _check(lib().mhd_set_stream(h, ptr))


def mhd_set_graphs(h, enable: bool):
    _check(lib().mhd_set_graphs(h, 1 if enable else 0))


def mhd_set_fusion(h, mode):
    """mode: 0 / False never, 1 / True where faster (default), 2 wherever it applies."""
    _check(lib().mhd_set_fusion(h, int(mode)))


def mhd_set_state(h, host_state: np.ndarray):
    a = np.ascontiguousarray(host_state)
    _check(lib().mhd_set_state(h, a.ctypes.data_as(ctypes.c_void_p)))


def mhd_set_state_device(h, dev_state):
    _check(lib().mhd_set_state_device(h, ctypes.c_void_p(_dev_ptr(dev_state))))


def mhd_get_state(h, out: np.ndarray):
    if not out.flags["C_CONTIGUOUS"]:
        raise ValueError("output array must be C-contiguous")
    _check(lib().mhd_get_state(h, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def mhd_get_state_device(h, dev_state):
    _check(lib().mhd_get_state_device(h, ctypes.c_void_p(_dev_ptr(dev_state))))


def mhd_step(h, n: int, cfl: float):
    _check(lib().mhd_step(h, n, cfl))


def mhd_divb_max(h) -> float:
    v = ctypes.c_double()
    _check(lib().mhd_divb_max(h, ctypes.byref(v)))
    return v.value


def mhd_divb_max_noalloc(dev_state, nx: int, ny: int, nz: int, bc: int, dtype: int, dev_out, stream=None):
    """dev_state / dev_out: device tensors (or raw device addresses); dev_out
    receives one double, asynchronously on `stream`."""
    sp = None if stream is None else (stream if isinstance(stream, int) else int(stream.cuda_stream))
    _check(lib().mhd_divb_max_noalloc(_dev_ptr(dev_state), nx, ny, nz, bc, dtype, _dev_ptr(dev_out), sp))


def mhd_get_time(h):
    t = ctypes.c_double()
    s = ctypes.c_int64()
    _check(lib().mhd_get_time(h, ctypes.byref(t), ctypes.byref(s)))
    return t.value, s.value


def mhd_set_time(h, t: float, s: int):
    _check(lib().mhd_set_time(h, t, s))


def mhd_set_stop_time(h, t_stop):
    _check(lib().mhd_set_stop_time(h, -1.0 if t_stop is None else float(t_stop)))


def mhd_fluid_sweep(h, axis: int, dt: float):
    _check(lib().mhd_fluid_sweep(h, axis, dt))


def mhd_ct_sweep(h, axis: int, dt: float):
    _check(lib().mhd_ct_sweep(h, axis, dt))


def mhd_cmax(h) -> float:
    v = ctypes.c_double()
    _check(lib().mhd_cmax(h, ctypes.byref(v)))
    return v.value


def mhd_step_dt(h, dt: float, s_order: int):
    _check(lib().mhd_step_dt(h, dt, s_order))


def mhd_state_bytes(nx: int, ny: int, nz: int, dtype: int) -> int:
    return int(lib().mhd_state_bytes(nx, ny, nz, dtype))


def mhd_workspace_bytes(nx: int, ny: int, nz: int, dtype: int) -> int:
    return int(lib().mhd_workspace_bytes(nx, ny, nz, dtype))


def mhd_bind_workspace(h, dev, nbytes: int):
    """dev: a device buffer (torch tensor or address) the caller keeps alive longer than the handle."""
    _check(lib().mhd_bind_workspace(h, ctypes.c_void_p(_dev_ptr(dev)), int(nbytes)))


def mhd_timing(h, enable: bool):
    _check(lib().mhd_timing(h, 1 if enable else 0))


def mhd_timing_read(h, kind: int):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().mhd_timing_read(h, kind, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def mhd_diagnostic(h, kind: int, axis: int, index: int, dev_out):
    """dev_out: a torch tensor on the GPU (or a raw device address) with room for the field."""
    _check(lib().mhd_diagnostic(h, kind, axis, index, ctypes.c_void_p(_dev_ptr(dev_out))))


def mhd_batch_create(dtype: int):
    h = ctypes.c_void_p()
    _check(lib().mhd_batch_create(dtype, ctypes.byref(h)))
    return h


def mhd_batch_destroy(b):
    _check(lib().mhd_batch_destroy(b))


def mhd_batch_set_stream(b, stream):
    ptr = None if stream is None else (stream if isinstance(stream, int) else int(stream.cuda_stream))
    _check(lib().mhd_batch_set_stream(b, ptr))


def mhd_batch_problem_bytes(nx: int, ny: int, nz: int, dtype: int) -> int:
    return int(lib().mhd_batch_problem_bytes(nx, ny, nz, dtype))


def mhd_batch_add(b, nx: int, ny: int, nz: int, gamma: float, bc: int, host_state: np.ndarray) -> int:
    a = np.ascontiguousarray(host_state)
    pid = ctypes.c_int()
    _check(lib().mhd_batch_add(b, nx, ny, nz, gamma, bc, a.ctypes.data_as(ctypes.c_void_p), ctypes.byref(pid)))
    return pid.value


def mhd_batch_add_device(b, nx: int, ny: int, nz: int, gamma: float, bc: int, dev_state) -> int:
    pid = ctypes.c_int()
    _check(lib().mhd_batch_add_device(b, nx, ny, nz, gamma, bc, ctypes.c_void_p(_dev_ptr(dev_state)),
                                      ctypes.byref(pid)))
    return pid.value


def mhd_batch_problem_layout(nx: int, ny: int, nz: int, dtype: int):
    """(offset of conserved fields copy 0, offset of face fields copy 0, offset of the control block, block bytes)."""
    v = [ctypes.c_size_t() for _ in range(4)]
    _check(lib().mhd_batch_problem_layout(nx, ny, nz, dtype, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


def mhd_batch_add_inplace(b, nx: int, ny: int, nz: int, gamma: float, bc: int, dev_block, ready=None) -> int:
    """dev_block: a device buffer (torch tensor or address) of mhd_batch_problem_bytes bytes holding the initial
    state at the copy-0 offsets; ready: a hipEvent_t address (or None)."""
    pid = ctypes.c_int()
    _check(lib().mhd_batch_add_inplace(b, nx, ny, nz, gamma, bc, ctypes.c_void_p(_dev_ptr(dev_block)),
                                       None if ready is None else ctypes.c_void_p(int(ready)), ctypes.byref(pid)))
    return pid.value


def mhd_batch_record(b, event):
    """event: a hipEvent_t address (e.g. torch.cuda.Event().cuda_event)."""
    _check(lib().mhd_batch_record(b, ctypes.c_void_p(int(event))))


def mhd_batch_remove(b, pid: int):
    _check(lib().mhd_batch_remove(b, pid))


def mhd_batch_count(b):
    n = ctypes.c_int()
    nbytes = ctypes.c_size_t()
    _check(lib().mhd_batch_count(b, ctypes.byref(n), ctypes.byref(nbytes)))
    return n.value, nbytes.value


def mhd_batch_step(b, n: int, cfl: float):
    _check(lib().mhd_batch_step(b, n, cfl))


def mhd_batch_get_state(b, pid: int, out: np.ndarray):
    if not out.flags["C_CONTIGUOUS"]:
        raise ValueError("output array must be C-contiguous")
    _check(lib().mhd_batch_get_state(b, pid, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def mhd_batch_get_state_device(b, pid: int, dev_state):
    _check(lib().mhd_batch_get_state_device(b, pid, ctypes.c_void_p(_dev_ptr(dev_state))))


def mhd_batch_get_time(b, pid: int):
    t = ctypes.c_double()
    s = ctypes.c_int64()
    _check(lib().mhd_batch_get_time(b, pid, ctypes.byref(t), ctypes.byref(s)))
    return t.value, s.value


def mhd_batch_set_stop_time(b, pid: int, t_stop):
    _check(lib().mhd_batch_set_stop_time(b, pid, -1.0 if t_stop is None else float(t_stop)))


def mhd_batch_status(b, pid: int) -> int:
    """MHD_OK or MHD_ERR_NONFINITE; other errors raise."""
    rc = lib().mhd_batch_status(b, pid)
    if rc not in (MHD_OK, MHD_ERR_NONFINITE):
        _check(rc)
    return rc


def mhd_batch_set_graphs(b, enable: bool):
    _check(lib().mhd_batch_set_graphs(b, 1 if enable else 0))


def mhd_batch_autotune(b, reps: int = 3):
    _check(lib().mhd_batch_autotune(b, reps))


def mhd_batch_set_tile(b, pid: int, kind: int, p0: int, p1: int = 0):
    _check(lib().mhd_batch_set_tile(b, pid, kind, p0, p1))


def mhd_batch_tile(b, pid: int, kind: int):
    p0 = ctypes.c_int()
    p1 = ctypes.c_int()
    _check(lib().mhd_batch_tile(b, pid, kind, ctypes.byref(p0), ctypes.byref(p1)))
    return p0.value, p1.value


MHD_REQ_QUEUED, MHD_REQ_RUNNING, MHD_REQ_DONE = 0, 1, 2


def mhd_server_now() -> float:
    return float(lib().mhd_server_now())


def mhd_server_create(hbm_budget: int, cfl: float):
    h = ctypes.c_void_p()
    _check(lib().mhd_server_create(int(hbm_budget), cfl, ctypes.byref(h)))
    return h


def mhd_server_destroy(s):
    _check(lib().mhd_server_destroy(s))


def mhd_server_set_max_cells(s, cells: int):
    _check(lib().mhd_server_set_max_cells(s, int(cells)))


def mhd_server_submit(s, nx: int, ny: int, nz: int, gamma: float, bc: int, dtype: int, host_state: np.ndarray,
                      nsteps: int) -> int:
    a = np.ascontiguousarray(host_state, dtype=_np_dtype(dtype))
    rid = ctypes.c_int()
    _check(lib().mhd_server_submit(s, nx, ny, nz, gamma, bc, dtype, a.ctypes.data_as(ctypes.c_void_p), nsteps,
                                   ctypes.byref(rid)))
    return rid.value


def mhd_server_submit_ref(s, nx: int, ny: int, nz: int, gamma: float, bc: int, dtype: int, host_state: np.ndarray,
                          nsteps: int) -> int:
    """Lend host_state (C-contiguous, of the request's dtype, no temporary copy is made) until the request
    leaves the queue; the caller keeps it alive and unchanged until then."""
    if not (isinstance(host_state, np.ndarray) and host_state.flags.c_contiguous
            and host_state.dtype == _np_dtype(dtype)):
        raise ValueError("a lent state must be a C-contiguous array of the request's dtype")
    rid = ctypes.c_int()
    _check(lib().mhd_server_submit_ref(s, nx, ny, nz, gamma, bc, dtype, host_state.ctypes.data_as(ctypes.c_void_p),
                                       nsteps, ctypes.byref(rid)))
    return rid.value


def mhd_server_tick(s):
    running = ctypes.c_int()
    queued = ctypes.c_int()
    _check(lib().mhd_server_tick(s, ctypes.byref(running), ctypes.byref(queued)))
    return running.value, queued.value


def mhd_server_poll(s) -> int:
    rid = ctypes.c_int()
    _check(lib().mhd_server_poll(s, ctypes.byref(rid)))
    return rid.value


def mhd_server_info(s, rid: int) -> dict:
    st, status = ctypes.c_int(), ctypes.c_int()
    t, ta, tb, tc = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().mhd_server_info(s, rid, ctypes.byref(st), ctypes.byref(t), ctypes.byref(n), ctypes.byref(status),
                                 ctypes.byref(ta), ctypes.byref(tb), ctypes.byref(tc)))
    return {"state": st.value, "t_sim": t.value, "steps": n.value, "status": status.value, "t_submit": ta.value,
            "t_admit": tb.value, "t_finish": tc.value}


def mhd_server_take(s, rid: int, out: np.ndarray):
    if not out.flags["C_CONTIGUOUS"]:
        raise ValueError("output array must be C-contiguous")
    _check(lib().mhd_server_take(s, rid, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def mhd_server_stats(s):
    nbytes = ctypes.c_size_t()
    cu = ctypes.c_int64()
    _check(lib().mhd_server_stats(s, ctypes.byref(nbytes), ctypes.byref(cu)))
    return nbytes.value, cu.value


class Server:
    """Owning wrapper of one request server (host-side convenience; no computation)."""

    def __init__(self, hbm_budget: int, cfl: float = 0.7, max_cells=None):
        self.s = mhd_server_create(hbm_budget, cfl)
        self.meta = {}
        self.lent = {}   # request id -> lent state, held until the request is taken
        if max_cells is not None:
            mhd_server_set_max_cells(self.s, max_cells)

    def close(self):
        if self.s is not None:
            mhd_server_destroy(self.s)
            self.s = None
        self.lent.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, state: np.ndarray, gamma: float, bc: int, dtype: int, nsteps: int, lend: bool = False) -> int:
        nz, ny, nx = state.shape[1:]
        if lend:
            rid = mhd_server_submit_ref(self.s, nx, ny, nz, gamma, bc, dtype, state, nsteps)
            self.lent[rid] = state
        else:
            rid = mhd_server_submit(self.s, nx, ny, nz, gamma, bc, dtype, state, nsteps)
        self.meta[rid] = (state.shape, dtype)
        return rid

    def tick(self):
        return mhd_server_tick(self.s)

    def finished(self):
        """Ids of requests finished since the last call."""
        out = []
        while True:
            rid = mhd_server_poll(self.s)
            if rid < 0:
                return out
            out.append(rid)

    def info(self, rid: int) -> dict:
        return mhd_server_info(self.s, rid)

    def take(self, rid: int) -> np.ndarray:
        shape, dtype = self.meta.pop(rid)
        out = np.empty(shape, dtype=_np_dtype(dtype))
        mhd_server_take(self.s, rid, out)
        self.lent.pop(rid, None)
        return out


class Batch:
    """Owning wrapper of one batch (host-side convenience; no computation)."""

    def __init__(self, dtype=MHD_F64):
        self.dtype = dtype
        self.np_dtype = _np_dtype(dtype)
        self.shapes = {}
        self.b = mhd_batch_create(dtype)

    def close(self):
        if self.b is not None:
            mhd_batch_destroy(self.b)
            self.b = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, state: np.ndarray, gamma: float, bc: int = MHD_BC_PERIODIC) -> int:
        a = np.ascontiguousarray(state, dtype=self.np_dtype)
        if a.ndim != 4 or a.shape[0] != 8:
            raise ValueError("state must have shape (8, nz, ny, nx)")
        nz, ny, nx = a.shape[1:]
        pid = mhd_batch_add(self.b, nx, ny, nz, gamma, bc, a)
        self.shapes[pid] = a.shape
        return pid

    def remove(self, pid: int):
        mhd_batch_remove(self.b, pid)
        self.shapes.pop(pid, None)

    def step(self, n: int = 1, cfl: float = 0.7):
        mhd_batch_step(self.b, n, cfl)

    def get_state(self, pid: int) -> np.ndarray:
        out = np.empty(self.shapes[pid], dtype=self.np_dtype)
        return mhd_batch_get_state(self.b, pid, out)

    def time(self, pid: int):
        return mhd_batch_get_time(self.b, pid)

    def status(self, pid: int) -> int:
        return mhd_batch_status(self.b, pid)

    def autotune(self, reps: int = 3):
        mhd_batch_autotune(self.b, reps)


class Solver:
    """Owning wrapper of one handle (host-side convenience; no computation)."""

    def __init__(self, nx, ny, nz, gamma, bc=MHD_BC_PERIODIC, dtype=MHD_F64):
        self.shape = (8, nz, ny, nx)
        self.dtype = dtype
        self.np_dtype = _np_dtype(dtype)
        self.h = mhd_create(nx, ny, nz, gamma, bc, dtype)

    def close(self):
        if self.h is not None:
            mhd_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, s: np.ndarray):
        a = np.ascontiguousarray(s, dtype=self.np_dtype)
        if a.size != int(np.prod(self.shape)):
            raise ValueError("state has %d elements, expected %d" % (a.size, int(np.prod(self.shape))))
        mhd_set_state(self.h, a)

    def get_state(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=self.np_dtype)
        return mhd_get_state(self.h, out)

    def step(self, n: int, cfl: float = 0.7):
        mhd_step(self.h, n, cfl)

    def run_to(self, t_stop: float, cfl: float = 0.7, max_steps: int = 1000000, chunk: int = 64):
        mhd_set_stop_time(self.h, t_stop)
        steps = 0
        while self.time()[0] < t_stop and steps < max_steps:
            mhd_step(self.h, chunk, cfl)
            steps += chunk

    def time(self):
        return mhd_get_time(self.h)

    def divb_max(self) -> float:
        return mhd_divb_max(self.h)

    def cmax(self) -> float:
        return mhd_cmax(self.h)

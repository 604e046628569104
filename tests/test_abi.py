"""CPU checks of the C ABI boundary: the built library loads, exports every
function the headers under include/ declare, and rejects bad arguments before
touching a device. No compute call is made here."""
from __future__ import annotations

import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**\s*(mhd_\w+)\s*\(", text, flags=re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def libmhd():
    from paper_0908_4362_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libmhd.so is not built (run python -m paper_0908_4362_amd.build)")
    return binding


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("mhd_create", "mhd_set_state", "mhd_step", "mhd_get_state", "mhd_divb_max", "mhd_destroy",
              "mhd_batch_create", "mhd_batch_add", "mhd_batch_step", "mhd_batch_get_state", "mhd_batch_autotune"):
        assert n in names
    assert len(names) >= 35


def test_library_exports_every_declared_symbol(libmhd):
    out = subprocess.run(["nm", "-D", "--defined-only", libmhd.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    L = libmhd.lib()
    for n in declared_functions():
        assert hasattr(L, n)


def test_binding_exposes_the_same_names(libmhd):
    for n in declared_functions():
        assert callable(getattr(libmhd, n)), n


def test_argument_errors_are_reported_before_device_use(libmhd):
    B = libmhd
    bad = [
        (0, 4, 4, 1.4, 0, B.MHD_F64),
        (4, -1, 4, 1.4, 0, B.MHD_F64),
        (4, 4, 4, 1.0, 0, B.MHD_F64),
        (4, 4, 4, float("nan"), 0, B.MHD_F64),
        (4, 4, 4, 1.4, 7, B.MHD_F64),
        (4, 4, 4, 1.4, 0, 5),
        (8192, 8192, 1025, 1.4, 0, B.MHD_F32),   # more than 2^36 cells
    ]
    for args in bad:
        with pytest.raises(B.MHDError) as ei:
            B.mhd_create(*args)
        assert ei.value.code == B.MHD_ERR_ARG
        assert B.mhd_last_error()
    h = ctypes.c_void_p()
    assert B.lib().mhd_create(4, 4, 4, 1.4, 0, 1, None) == B.MHD_ERR_ARG
    assert B.lib().mhd_step(None, 1, 0.7) == B.MHD_ERR_ARG
    assert B.lib().mhd_destroy(None) == B.MHD_OK
    assert B.mhd_state_bytes(0, 1, 1, B.MHD_F32) == 0
    assert B.mhd_state_bytes(4, 4, 4, B.MHD_F32) >= 2 * 8 * 64 * 4
    assert B.mhd_state_bytes(8192, 8192, 1025, B.MHD_F32) == 0
    assert h.value is None


def test_batch_argument_errors_are_reported_before_device_use(libmhd):
    B = libmhd
    L = B.lib()
    out = ctypes.c_void_p()
    assert L.mhd_batch_create(7, ctypes.byref(out)) == B.MHD_ERR_ARG and out.value is None
    assert L.mhd_batch_create(B.MHD_F64, None) == B.MHD_ERR_ARG
    assert L.mhd_batch_destroy(None) == B.MHD_OK
    pid = ctypes.c_int()
    assert L.mhd_batch_add(None, 4, 4, 4, 1.4, 0, None, ctypes.byref(pid)) == B.MHD_ERR_ARG
    assert L.mhd_batch_step(None, 1, 0.7) == B.MHD_ERR_ARG
    assert L.mhd_batch_remove(None, 1) == B.MHD_ERR_ARG
    assert L.mhd_batch_status(None, 1) == B.MHD_ERR_ARG
    assert L.mhd_batch_autotune(None, 1) == B.MHD_ERR_ARG
    assert B.mhd_batch_problem_bytes(0, 4, 4, B.MHD_F64) == 0
    assert B.mhd_batch_problem_bytes(4, 4, 4, 3) == 0
    assert B.mhd_batch_problem_bytes(8192, 8192, 1025, B.MHD_F32) == 0   # more than 2^36 cells
    # two state copies of 8 fields, control block and reduction slots
    for (nx, ny, nz) in ((32, 32, 32), (48, 20, 7), (128, 1, 1)):
        for dt, es in ((B.MHD_F32, 4), (B.MHD_F64, 8)):
            nbytes = B.mhd_batch_problem_bytes(nx, ny, nz, dt)
            assert 16 * nx * ny * nz * es < nbytes < 16 * nx * ny * nz * es + 6 * 256 + 8 * 65536


def test_workspace_bytes(libmhd):
    B = libmhd
    assert B.mhd_workspace_bytes(0, 4, 4, B.MHD_F64) == 0
    assert B.mhd_workspace_bytes(4, 4, 4, 9) == 0
    for (nx, ny, nz) in ((32, 32, 32), (50, 7, 3), (256, 1, 1)):
        for dt, es in ((B.MHD_F32, 4), (B.MHD_F64, 8)):
            nb = B.mhd_workspace_bytes(nx, ny, nz, dt)
            assert nb % 256 == 0 and nb >= 16 * nx * ny * nz * es
            assert B.mhd_state_bytes(nx, ny, nz, dt) == nb

"""CPU checks of the C ABI boundary: the built library loads, exports every
function include/mhd.h declares, and rejects bad arguments before touching a
device. No compute call is made here."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**\s*(mhd_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def libmhd():
    from paper_0908_4362_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        pytest.fail("libmhd.so is not built (run python -m paper_0908_4362_amd.build)")
    return binding


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("mhd_create", "mhd_set_state", "mhd_step", "mhd_get_state", "mhd_divb_max", "mhd_destroy"):
        assert n in names
    assert len(names) >= 18


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
    assert h.value is None

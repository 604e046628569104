"""GPU checks of the headless diagnostics (mhd_diagnostic): each derived field
against the same formula evaluated with numpy on the host copy of the state,
and every plane equal to the matching plane of the whole-grid field."""
from __future__ import annotations

import numpy as np
import pytest

from paper_0908_4362_amd import problems as P
from tests import helpers as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_4362_amd import binding

    binding.lib()
    return binding


def reference(s, gamma, bc):
    """Derived fields of a state (8, nz, ny, nx) in float64."""
    s = s.astype(np.float64)

    def up(a, axis):   # value on the upper face: next cell's lower face through the boundary map
        if bc == 0:
            return np.roll(a, -1, axis=axis)
        idx = [slice(None)] * 3
        out = np.roll(a, -1, axis=axis)
        idx[axis] = -1
        out[tuple(idx)] = a[tuple(idx)]
        return out

    bx = 0.5 * (s[5] + up(s[5], 2))
    by = 0.5 * (s[6] + up(s[6], 1))
    bz = 0.5 * (s[7] + up(s[7], 0))
    bb = bx * bx + by * by + bz * bz
    rho = s[0]
    v = [s[1 + a] / rho for a in range(3)]
    vv = v[0] ** 2 + v[1] ** 2 + v[2] ** 2
    p = (gamma - 1.0) * (s[4] - 0.5 * rho * vv - 0.5 * bb)
    div = (up(s[5], 2) - s[5]) + (up(s[6], 1) - s[6]) + (up(s[7], 0) - s[7])
    vm = np.maximum(np.abs(v[0]), np.maximum(np.abs(v[1]), np.abs(v[2])))
    return [p, 0.5 * bb, np.sqrt(vv), div, vm + np.sqrt(np.abs(gamma * p + bb) / rho)]


@pytest.mark.parametrize("dtype,bc", [(1, 0), (1, 1), (0, 0)])
def test_diagnostics_match_numpy(B, dtype, bc):
    import torch

    nx, ny, nz = 30, 22, 18
    s = P.random_smooth(nx, ny, nz, seed=P.MASTER_SEED + 700)
    tdt = torch.float64 if dtype == 1 else torch.float32
    with B.Solver(nx, ny, nz, H.GAMMA53, bc, dtype) as sv:
        sv.set_state(s)
        sv.step(2)
        st = sv.get_state()
        ref = reference(st, H.GAMMA53, bc)
        for kind in range(B.MHD_D_COUNT):
            full = torch.empty(nx * ny * nz, dtype=tdt, device="cuda")
            B.mhd_diagnostic(sv.h, kind, -1, 0, full)
            torch.cuda.synchronize()
            got = full.cpu().numpy().astype(np.float64).reshape(nz, ny, nx)
            want = ref[kind]
            scale = max(np.abs(want).max(), 1e-300) if kind != B.MHD_D_DIVB else 1.0
            tol = 1e-13 if dtype == 1 else 2e-6
            if kind == B.MHD_D_DIVB:
                tol = 1e-13 if dtype == 1 else 1e-5
            assert np.abs(got - want).max() <= tol * scale, kind
            # planes equal the matching planes of the whole-grid field
            for axis, idx in ((0, 7), (1, ny - 1), (2, 0), (2, nz - 1)):
                npl = {0: ny * nz, 1: nx * nz, 2: nx * ny}[axis]
                pl = torch.empty(npl, dtype=tdt, device="cuda")
                B.mhd_diagnostic(sv.h, kind, axis, idx, pl)
                torch.cuda.synchronize()
                f3 = full.cpu().numpy().reshape(nz, ny, nx)
                plane = f3[:, :, idx] if axis == 0 else (f3[:, idx, :] if axis == 1 else f3[idx])
                assert np.array_equal(pl.cpu().numpy().reshape(plane.shape), plane), (kind, axis, idx)


def test_diagnostic_argument_errors(B):
    import torch

    out = torch.empty(64, dtype=torch.float64, device="cuda")
    with B.Solver(4, 4, 4, H.GAMMA53) as sv:
        sv.set_state(P.uniform(4, 4, 4, bvec=(0.1, 0.2, 0.3)))
        for bad in ((5, -1, 0), (-1, -1, 0), (0, 3, 0), (0, 0, 4), (0, 2, -1)):
            with pytest.raises(B.MHDError) as ei:
                B.mhd_diagnostic(sv.h, *bad, out)
            assert ei.value.code == B.MHD_ERR_ARG
        with pytest.raises(B.MHDError):
            B.mhd_diagnostic(sv.h, 0, -1, 0, 0)

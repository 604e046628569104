"""Parity at the benchmark's full size (256^3, the launch configuration bench.py
times): one full step of the blast wave from its initial state on the GPU,
checked on sampled 16^3 blocks that the oracle computes from 48^3 windows of
the same initial state (one step depends on cells at most 16 away, so the
window edges do not reach the compared block); plus properties that hold at
any size (conservation, div B) over several steps."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_0908_4362_amd import problems as P
from tests import helpers as H

pytestmark = pytest.mark.gpu

N = 256
WIN = 48
BLK = 16
CENTRES = [(128 + 25, 128, 128), (128, 128 - 25, 128), (128 + 18, 128 + 18, 128 - 3), (128, 128, 128 + 26),
           (20, 200, 77)]


@pytest.fixture(scope="module")
def B():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0908_4362_amd import binding

    binding.lib()
    return binding


def note(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


def window(s, c, w):
    idx = [np.arange(c[a] - w // 2, c[a] - w // 2 + w) % N for a in range(3)]
    return np.ascontiguousarray(s[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]]), idx


@pytest.fixture(scope="module")
def blast_ref(orc):
    s0 = P.blast(N)
    g = orc.Grid(N, N, N, H.GAMMA53)
    cmax = orc.cmax(g, s0)
    dt, _ = orc.dt_rule(cmax, 0.7, 0.0, None)
    blocks = []
    gw = orc.Grid(WIN, WIN, WIN, H.GAMMA53, orc.OUTFLOW)
    lo = WIN // 2 - BLK // 2
    for c in CENTRES:
        win, idx = window(s0, c, WIN)
        out = orc.step_dt(gw, win, dt, 0)
        blocks.append((out[:, lo:lo + BLK, lo:lo + BLK, lo:lo + BLK],
                       [i[lo:lo + BLK] for i in idx]))
    return s0, cmax, blocks


def gpu_block(st, idx):
    return st[:, idx[2]][:, :, idx[1]][:, :, :, idx[0]].astype(np.float64)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_blast_256_one_step_sampled(B, blast_ref, dtype):
    s0, cmax, blocks = blast_ref
    dt_code = B.MHD_F64 if dtype == "f64" else B.MHD_F32
    note("blast 256^3 %s one step" % dtype)
    with B.Solver(N, N, N, H.GAMMA53, 0, dt_code) as sv:
        sv.set_state(s0)
        assert sv.cmax() == pytest.approx(cmax, rel=1e-14 if dtype == "f64" else 1e-6)
        sv.step(1, 0.7)
        st = sv.get_state()
    worst = 0.0
    for (want, idx), c in zip(blocks, CENTRES):
        got = gpu_block(st, idx)
        if dtype == "f64":
            for f in range(8):
                assert H.rel_linf(got[f], want[f]) <= 1e-10, (c, f)
        else:
            # whole state of the block, so that a field that is nearly zero
            # there (a momentum component on a symmetry plane) is measured
            # against the size of the state, not against its own tiny values
            worst = max(worst, H.rel_l1(got, want))
    if dtype == "f32":
        # a shock problem: the FP32 error is reported and only gated against
        # gross mistakes (single-precision rounding can flip the upwind choice
        # at the exact ties this symmetric problem produces)
        note("blast 256^3 fp32 vs fp64 oracle, one step: worst rel L1 of a block %.2e" % worst)
        assert worst <= 1e-4


def test_blast_256_invariants(B):
    s0 = P.blast(N)
    note("blast 256^3 fp64 invariants 5 steps")
    with B.Solver(N, N, N, H.GAMMA53, 0, B.MHD_F64) as sv:
        sv.set_state(s0)
        d0 = sv.divb_max()
        sv.step(5, 0.7)
        st = sv.get_state()
        d1 = sv.divb_max()
    assert d0 == 0.0
    assert d1 <= 1e-12 * np.abs(st[5:]).max()
    for f in range(8):
        tot0 = np.sum(s0[f])
        scale = max(np.abs(s0[f]).sum(), np.abs(st[f]).sum())
        assert abs(np.sum(st[f]) - tot0) <= 1e-12 * scale, f

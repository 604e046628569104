"""GPU checks of batched solves (include/mhd_batch.h): every problem of a
batch must come out bitwise equal to a plain single-problem solve of the same
input and step count (the batched launches run the same kernel bodies), for
uneven grid sizes, both boundary conditions, both precisions, problems added
and removed between steps (cohorts in different sweep orders), graph replay,
autotuned tiles and a problem that fails alone. FP64 problems are also held
to the oracle gate (relative L-infinity <= 1e-10 per field)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

from paper_0908_4362_amd import problems as P
from tests import helpers as H

pytestmark = pytest.mark.gpu

F64_STEP_TOL = 1e-10


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


def plain(B, s, gamma, bc, dtype, nsteps, cfl=0.7, t_stop=None):
    nz, ny, nx = s.shape[1:]
    with B.Solver(nx, ny, nz, gamma, bc, dtype) as sv:
        sv.set_state(s)
        if t_stop is not None:
            B.mhd_set_stop_time(sv.h, t_stop)
        if nsteps:
            sv.step(nsteps, cfl)
        return sv.get_state(), sv.time()


def mixed_problems():
    """(state, gamma, bc): uneven sizes spanning several tiles and ragged
    tails, 1D / 2D / 3D, periodic and outflow, smooth and shocked."""
    seed = P.MASTER_SEED + 300
    return [
        (P.random_smooth(24, 20, 18, seed=seed), H.GAMMA53, 0),
        (P.random_smooth(33, 26, 20, seed=seed + 1), H.GAMMA53, 1),
        (P.blast(16), H.GAMMA53, 0),
        (P.random_smooth(70, 12, 9, seed=seed + 2), H.GAMMA53, 0),
        (P.brio_wu(96), 2.0, 1),
        (P.orszag_tang(32), H.GAMMA53, 0),
        (P.random_smooth(9, 67, 5, seed=seed + 3), 1.4, 1),
    ]


@pytest.mark.parametrize("dtype", [1, 0])
def test_batch_equals_plain_bitwise(B, dtype):
    probs = mixed_problems()
    note("batch of %d problems, dtype %d" % (len(probs), dtype))
    with B.Batch(dtype) as bt:
        ids = [bt.add(s, gm, bc) for (s, gm, bc) in probs]
        bt.step(5)
        for pid, (s, gm, bc) in zip(ids, probs):
            want, tw = plain(B, s, gm, bc, dtype, 5)
            got = bt.get_state(pid)
            assert np.array_equal(got, want), (pid, s.shape)
            assert bt.time(pid) == tw
            assert bt.status(pid) == B.MHD_OK


def test_batch_alfven_fp32_matches_oracle(B, orc):
    """Problems of the batched Alfven workload (its generator and sizes 32^3
    and 48^3), FP32 in one batch against the FP64 oracle after 10 steps. The
    fields with a unit background (rho, E, B) meet the smooth-problem FP32
    gate, relative L1 <= 1e-5. The momenta are the wave alone (amplitude
    1e-4 to 1e-2): their fluxes difference O(1) products (b_d b_e, P*) whose
    FP32 rounding is a fixed absolute floor, so their error relative to the
    wave grows as the amplitude shrinks; it is reported and bounded loosely."""
    specs = [sp for sp in P.alfven_batch_specs(40) if sp["n"] in (32, 48)][:3]
    note("alfven batch fp32 vs oracle, sizes %s" % [sp["n"] for sp in specs])
    with B.Batch(B.MHD_F32) as bt:
        states = [P.alfven_111(sp["n"], sp["b0"], sp["amp"], sp["gamma"]) for sp in specs]
        ids = [bt.add(st, sp["gamma"], 0) for st, sp in zip(states, specs)]
        bt.step(10)
        for pid, st, sp in zip(ids, states, specs):
            n = sp["n"]
            want, _, _ = orc.run(orc.Grid(n, n, n, sp["gamma"], 0), st, 10, 0.7)
            got = bt.get_state(pid).astype(np.float64)
            errs = [H.rel_l1(got[f], want[f]) for f in range(8)]
            note("n %d amp %.1e: FP32 rel L1 per field %s" % (n, sp["amp"], " ".join("%.1e" % e for e in errs)))
            assert max(errs[f] for f in (0, 4, 5, 6, 7)) <= 1e-5
            assert max(errs[1:4]) <= 5e-2


def test_batch_fp64_matches_oracle(B, orc):
    probs = mixed_problems()[:3]
    note("batch vs oracle")
    with B.Batch(B.MHD_F64) as bt:
        ids = [bt.add(s, gm, bc) for (s, gm, bc) in probs]
        bt.step(10)
        for pid, (s, gm, bc) in zip(ids, probs):
            nz, ny, nx = s.shape[1:]
            want, _, _ = orc.run(orc.Grid(nx, ny, nz, gm, bc), s, 10, 0.7)
            got = bt.get_state(pid)
            for f in range(8):
                assert H.rel_linf(got[f], want[f]) <= F64_STEP_TOL, (pid, f)


@pytest.mark.parametrize("graphs", [True, False])
def test_batch_staggered_admission(B, graphs):
    """Problems join and leave between steps; those that joined at different
    steps run different sweep orders in the same batched step."""
    seed = P.MASTER_SEED + 310
    a = P.random_smooth(20, 18, 16, seed=seed)
    b = P.random_smooth(28, 14, 22, seed=seed + 1)
    c = P.blast(20)
    d = P.random_smooth(17, 23, 11, seed=seed + 2)
    note("staggered admission, graphs %s" % graphs)
    with B.Batch(B.MHD_F64) as bt:
        B.mhd_batch_set_graphs(bt.b, graphs)
        ia = bt.add(a, H.GAMMA53, 0)
        bt.step(2)
        ib = bt.add(b, H.GAMMA53, 1)
        bt.step(3)
        assert np.array_equal(bt.get_state(ia), plain(B, a, H.GAMMA53, 0, 1, 5)[0])
        bt.remove(ia)
        ic = bt.add(c, H.GAMMA53, 0)
        bt.step(1)
        idd = bt.add(d, 1.4, 0)
        bt.step(4)
        assert B.mhd_batch_count(bt.b)[0] == 3
        for pid, (s, gm, bc, n) in ((ib, (b, H.GAMMA53, 1, 8)), (ic, (c, H.GAMMA53, 0, 5)), (idd, (d, 1.4, 0, 4))):
            want, tw = plain(B, s, gm, bc, 1, n)
            assert bt.time(pid)[1] == n
            assert np.array_equal(bt.get_state(pid), want), pid
            assert bt.time(pid) == tw


def test_batch_graph_replay_equals_eager(B):
    probs = mixed_problems()
    note("graph replay vs eager")
    out = []
    for graphs in (True, False):
        with B.Batch(B.MHD_F32) as bt:
            B.mhd_batch_set_graphs(bt.b, graphs)
            ids = [bt.add(s, gm, bc) for (s, gm, bc) in probs]
            for _ in range(7):   # every sweep order replayed at least twice
                bt.step(1)
            out.append([bt.get_state(pid) for pid in ids])
    for g, e in zip(*out):
        assert np.array_equal(g, e)


@pytest.mark.parametrize("dtype", [1, 0])
def test_batch_autotune_keeps_results(B, dtype):
    """Autotuned chunk lengths differ from the plain solve's; results may not
    (in FP32 too: FMA contraction stays within one expression, so the unrolled
    marching loop rounds every cell the same wherever its chunk starts)."""
    probs = mixed_problems()
    note("autotune, dtype %d" % dtype)
    with B.Batch(dtype) as bt:
        ids = [bt.add(s, gm, bc) for (s, gm, bc) in probs]
        bt.step(2)
        bt.autotune(2)
        for pid, (s, gm, bc) in zip(ids, probs):
            nz, ny, nx = s.shape[1:]
            for kind in range(1, B.MHD_K_CTFLUID_Z + 1):
                p0, p1 = B.mhd_batch_tile(bt.b, pid, kind)
                if kind in (B.MHD_K_FLUID_X, B.MHD_K_CT_X, B.MHD_K_CTFLUID_X):
                    # wavefront form (0, 0), or on FP32 periodic rows the lane-row form
                    # (K cells per lane, W lanes per row) where the row length has one
                    shape = {64: (1, 64), 128: (2, 64), 32: (1, 32), 96: (3, 32), 48: (3, 16)}.get(nx)
                    lrow = dtype == B.MHD_F32 and bc == 0 and shape is not None
                    assert (p0, p1) in ((0, 0), shape) if lrow else (p0, p1) == (0, 0)
                else:
                    axis = 1 if kind in (B.MHD_K_FLUID_Y, B.MHD_K_CT_Y, B.MHD_K_CTFLUID_Y) else 2
                    assert p0 <= s.shape[3 - axis]
        bt.step(3)
        for pid, (s, gm, bc) in zip(ids, probs):
            assert np.array_equal(bt.get_state(pid), plain(B, s, gm, bc, dtype, 5)[0]), pid


def test_batch_failure_is_isolated(B):
    seed = P.MASTER_SEED + 320
    good = P.random_smooth(22, 19, 13, seed=seed)
    bad = P.random_smooth(18, 18, 18, seed=seed + 1)
    bad[0, 3, 4, 5] = np.nan
    stall = P.uniform(14, 12, 10, rho=1.0, p=0.0)   # valid, but no positive wave speed
    note("failure isolation")
    with B.Batch(B.MHD_F64) as bt:
        ig = bt.add(good, H.GAMMA53, 0)
        with pytest.raises(B.MHDError) as ei:
            bt.add(bad, H.GAMMA53, 0)
        assert ei.value.code == B.MHD_ERR_ARG
        assert B.mhd_batch_count(bt.b)[0] == 1
        iz = bt.add(stall, H.GAMMA53, 0)
        bt.step(3)
        assert bt.status(iz) == B.MHD_ERR_NONFINITE
        assert np.array_equal(bt.get_state(iz), stall)
        assert bt.status(ig) == B.MHD_OK
        assert np.array_equal(bt.get_state(ig), plain(B, good, H.GAMMA53, 0, 1, 3)[0])


def test_batch_stop_time_per_problem(B):
    s1 = P.brio_wu(128)
    s2 = P.random_smooth(16, 16, 16, seed=P.MASTER_SEED + 330)
    note("per-problem stop time")
    with B.Batch(B.MHD_F64) as bt:
        i1 = bt.add(s1, 2.0, 1)
        i2 = bt.add(s2, H.GAMMA53, 0)
        B.mhd_batch_set_stop_time(bt.b, i1, 5.5)
        bt.step(60)
        assert bt.time(i1)[0] == 5.5
        want, tw = plain(B, s1, 2.0, 1, 1, 60, t_stop=5.5)
        assert np.array_equal(bt.get_state(i1), want)
        assert bt.time(i2) == plain(B, s2, H.GAMMA53, 0, 1, 60)[1]


def test_batch_device_input_equals_host_input(B):
    import torch

    s = P.random_smooth(30, 22, 18, seed=P.MASTER_SEED + 340)
    dev = torch.from_numpy(s).cuda()
    torch.cuda.synchronize()
    note("device input")
    with B.Batch(B.MHD_F64) as bt:
        i1 = B.mhd_batch_add_device(bt.b, 30, 22, 18, H.GAMMA53, 0, dev)
        bt.shapes[i1] = s.shape
        i2 = bt.add(s, H.GAMMA53, 0)
        bt.step(2)
        out = torch.empty_like(dev)
        B.mhd_batch_get_state_device(bt.b, i1, out)
        got = bt.get_state(i2)
        assert np.array_equal(bt.get_state(i1), got)
        torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), got)


def test_batch_argument_errors(B):
    with B.Batch(B.MHD_F64) as bt:
        with pytest.raises(B.MHDError) as ei:
            B.mhd_batch_add(bt.b, 0, 4, 4, 1.4, 0, np.zeros(8))
        assert ei.value.code == B.MHD_ERR_ARG
        with pytest.raises(B.MHDError):
            B.mhd_batch_remove(bt.b, 12345)
        with pytest.raises(B.MHDError):
            B.mhd_batch_step(bt.b, 1, 1.5)
        with pytest.raises(B.MHDError):
            B.mhd_batch_autotune(bt.b, 0)
        bt.step(2)   # an empty batch steps nothing


@pytest.mark.parametrize("dtype", [1, 0])
def test_batch_of_random_shapes_equals_plain_bitwise(B, dtype):
    """Thirty problems of seeded random shapes (1 to 90 cells per axis, so
    single cells, lines, planes and boxes with ragged tiles), boundary
    conditions and gamma in one batch, stepped in two bursts with problems
    joining in between: every one bitwise equal to its plain solve."""
    rng = np.random.Generator(np.random.PCG64(P.MASTER_SEED + 350 + dtype))
    probs = []
    for k in range(30):
        shape = [int(x) for x in rng.integers(1, 91, size=3)]
        shape[int(rng.integers(0, 3))] = int(rng.integers(1, 6))    # one short axis keeps the batch small
        nx, ny, nz = shape
        probs.append((P.random_smooth(nx, ny, nz, seed=P.MASTER_SEED + 360 + k), float(rng.choice([1.4, H.GAMMA53, 2.0])),
                      int(rng.integers(0, 2))))
    note("batch of %d random shapes, dtype %d" % (len(probs), dtype))
    with B.Batch(dtype) as bt:
        first = [bt.add(s, gm, bc) for (s, gm, bc) in probs[:20]]
        bt.step(2)
        later = [bt.add(s, gm, bc) for (s, gm, bc) in probs[20:]]
        bt.step(3)
        for pid, (s, gm, bc), n in [(p, q, 5) for p, q in zip(first, probs[:20])] + \
                                   [(p, q, 3) for p, q in zip(later, probs[20:])]:
            want, tw = plain(B, s, gm, bc, dtype, n)
            assert np.array_equal(bt.get_state(pid), want), (pid, s.shape)
            assert bt.time(pid) == tw


@pytest.mark.parametrize("dtype", [1, 0])
def test_flat_axes_match_the_marching_field_sweep(B, dtype):
    """Plain solves update the field along an axis of one cell in closed form
    (one thread per cell); batched solves keep the marching pipeline there.
    Planes and lines in every orientation, both boundary conditions, six full
    steps (each sweep order twice): the two bitwise equal."""
    shapes = [(37, 29, 1), (41, 1, 23), (1, 19, 27), (53, 1, 1), (1, 31, 1), (1, 1, 29), (70, 1, 3)]
    probs = [(P.random_smooth(nx, ny, nz, seed=P.MASTER_SEED + 380 + k), H.GAMMA53, k % 2)
             for k, (nx, ny, nz) in enumerate(shapes)]
    note("flat-axis shapes, dtype %d" % dtype)
    with B.Batch(dtype) as bt:
        ids = [bt.add(s, gm, bc) for (s, gm, bc) in probs]
        bt.step(6)
        for pid, (s, gm, bc) in zip(ids, probs):
            want, tw = plain(B, s, gm, bc, dtype, 6)
            assert np.array_equal(bt.get_state(pid), want), s.shape
            assert bt.time(pid) == tw


@pytest.mark.parametrize("nx", [32, 48, 64, 96, 128, 192, 256])
def test_lane_row_x_sweeps_equal_batched_wavefront_form(B, nx):
    """A plain FP32 handle on periodic rows of 64 k cells (a whole row per
    wavefront) or of 32, 48 and 96 cells (two or four rows per wavefront) runs
    the x sweeps in the lane-row form and the reverse L_x fused; a batch whose
    x sweeps (the fused reverse one included) are pinned to the wavefront form
    (the autotuner's other candidate) runs the wavefront-form bodies. Both
    must give the same bits, with fusion on and off, after steps in all three
    sweep orders; so must the batch with its default tiles (the lane-row form
    on rows of 32, 48, 64, 96 and 128 cells)."""
    ny, nz = 11, 6
    s = P.random_smooth(nx, ny, nz, seed=P.MASTER_SEED + 340 + nx)
    note("lane-row x sweeps, %d x %d x %d fp32" % (nx, ny, nz))
    with B.Batch(B.MHD_F32) as bt:
        pid = bt.add(s, H.GAMMA53, 0)
        bt.step(4)
        dflt = bt.get_state(pid)
    with B.Batch(B.MHD_F32) as bt:
        pid = bt.add(s, H.GAMMA53, 0)
        B.mhd_batch_set_tile(bt.b, pid, B.MHD_K_FLUID_X, 0)
        B.mhd_batch_set_tile(bt.b, pid, B.MHD_K_CT_X, 0)
        B.mhd_batch_set_tile(bt.b, pid, B.MHD_K_CTFLUID_X, 0)
        with pytest.raises(B.MHDError):
            B.mhd_batch_set_tile(bt.b, pid, B.MHD_K_CT_X, 3)   # not a candidate
        bt.step(4)
        want = bt.get_state(pid)
    assert np.array_equal(dflt, want)
    for fusion in (1, 0):
        with B.Solver(nx, ny, nz, H.GAMMA53, 0, B.MHD_F32) as sv:
            B.mhd_set_fusion(sv.h, fusion)
            sv.set_state(s)
            sv.step(4)
            assert np.array_equal(sv.get_state(), want), fusion


@pytest.mark.parametrize("dtype,flat", [(0, False), (0, True), (1, False)])
def test_batch_fused_reverse_sweeps_equal_two_launches(B, dtype, flat):
    """A cohort of periodic problems runs each reverse L_d as one fused
    launch (field update, then fluid update) where every member has more than
    one cell along d; a plane in the cohort keeps the two launches along its
    short axis. Six full steps (each sweep order twice) with the default
    tiles, then with the fused tiles pinned to the shortest chunk along y and
    z and the wavefront form along x: every problem bitwise equal to a plain
    solve with fusion off."""
    shapes = [(24, 20, 18), (70, 12, 9), (64, 10, 7), (128, 6, 5), (33, 29, 3), (5, 7, 9), (18, 60, 31)]
    if flat:
        shapes.append((40, 36, 1))
    probs = [P.random_smooth(nx, ny, nz, seed=P.MASTER_SEED + 390 + k) for k, (nx, ny, nz) in enumerate(shapes)]
    note("fused reverse sweeps in a batch, dtype %d, plane %s" % (dtype, flat))
    wants = []
    for s in probs:
        nz, ny, nx = s.shape[1:]
        with B.Solver(nx, ny, nz, H.GAMMA53, 0, dtype) as sv:
            B.mhd_set_fusion(sv.h, 0)
            sv.set_state(s)
            sv.step(6)
            wants.append((sv.get_state(), sv.time()))
    for pin in (False, True):
        with B.Batch(dtype) as bt:
            ids = [bt.add(s, H.GAMMA53, 0) for s in probs]
            if pin:
                for pid, s in zip(ids, probs):
                    nz, ny, nx = s.shape[1:]
                    B.mhd_batch_set_tile(bt.b, pid, B.MHD_K_CTFLUID_X, 0)
                    for kind, n in ((B.MHD_K_CTFLUID_Y, ny), (B.MHD_K_CTFLUID_Z, nz)):
                        p0, _ = B.mhd_batch_tile(bt.b, pid, kind)
                        for c in ((n + 7) // 8, (n + 3) // 4, (n + 1) // 2):
                            if c >= 14 and c < p0:
                                B.mhd_batch_set_tile(bt.b, pid, kind, c)
                                break
            bt.step(6)
            for pid, s, (want, tw) in zip(ids, probs, wants):
                assert np.array_equal(bt.get_state(pid), want), (pin, s.shape)
                assert bt.time(pid) == tw

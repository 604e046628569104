#!/usr/bin/env python3
"""Benchmark of the MHD time step on one MI355X.

Workload: the 3D MHD blast wave on a periodic 256^3 unit cube (gamma = 5/3,
rho = 1, p = 10 inside r < 0.1 about the centre and 0.1 outside, uniform
B = (1/sqrt2, 1/sqrt2, 0), v = 0), CFL 0.7, W warm-up steps then K timed full
steps. A full step is the CFL reduction plus the forward and reverse sweeps
(12 directional sub-operations) and advances t by 2 dt. The state is resident
in HBM before the timed region; the whole step runs in the HIP library.

Prints one JSON line: cell-updates/s per full step (FP64 headline, FP32 next
to it; the K steps run as the library runs them, replayed from HIP graphs on
a stream of their own), the roofline of the dominant kernel from HIP events
recorded around every launch on the handle's stream during K further timed
steps (the events keep those steps out of graph replay and add about 3 %, so
they are not in the headline pass), the CPU oracle timed on a bounded
sample of the same workload, and the batched workload (many periodic linear
Alfven waves of sizes drawn from {32, 48, 64, 96, 128}^3, FP32, advanced
together by the batch runtime) against looping the plain solver over the same
problems, with a bitwise comparison of every final state; and the serving
workload (seeded requests for blast waves and extruded Orszag-Tang vortices of
32^3 to 192^3 cells, FP32 or FP64, 100 steps each, Poisson arrivals at
fractions of the measured saturation rate, admitted under an HBM budget)
against a first-come first-served queue of plain solves with the same
arrivals.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import platform
import sys
import time

HBM_PEAK_GBS = 8000.0
# algorithmic words per cell of one launch of each kernel kind: fluid_d reads rho, m, E and the three face fields and writes rho, m, E; the
# field update reads rho, m_d and the three face fields and writes the face
# fields; the CFL reduction reads all eight fields.
# a fused reverse L_d (field update, then fluid update, in one launch) reads the 8 fields and writes them.
WORDS_PER_CELL = {"cfl": 8, "fluid_x": 13, "fluid_y": 13, "fluid_z": 13, "ct_x": 8, "ct_y": 8, "ct_z": 8,
                  "ctfluid_x": 16, "ctfluid_y": 16, "ctfluid_z": 16}
STEP_WORDS = 104  # minimum per full step: 6 directional operators x (8 read + 8 written) + 8 for the CFL


def repeat_summary(reps, steps):
    """Per-step times of the repeated K-step passes (after the headline pass) and their median."""
    if not reps:
        return None
    ms = sorted(r * 1e3 / steps for r in reps)
    mid = len(ms) // 2
    med = ms[mid] if len(ms) % 2 else 0.5 * (ms[mid - 1] + ms[mid])
    return {"passes": len(ms), "steps_each": steps, "median_ms_per_step": round(med, 4),
            "min_ms_per_step": round(ms[0], 4), "max_ms_per_step": round(ms[-1], 4)}


def design_step_words(kern, steps):
    """Words per cell per full step of the launches the step ran (the instrumented pass's launch
    counts times each kind's words; the c_max reduction rides on the last fluid launch of the previous
    step, so only the dt finisher, which reads no cells, is counted under cfl)."""
    total = 0.0
    for k, (ms, cnt) in kern.items():
        if k != "cfl":
            total += WORDS_PER_CELL[k] * cnt
    return round(total / max(1, steps), 2)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def run_gpu(B, P, n, dtype, warmup, steps, stream, repeats=5):
    """W warm-up steps; then the headline pass, K full steps timed by the host clock between device
    synchronisations; then the instrumented pass, K more full steps with a HIP event pair around every
    launch (mhd_timing), whose per-kernel averages feed the roofline; then `repeats` more passes of K
    full steps timed like the headline (their median is reported beside it)."""
    nx = ny = nz = n
    sv = B.Solver(nx, ny, nz, 5.0 / 3.0, B.MHD_BC_PERIODIC, dtype)
    B.mhd_set_stream(sv.h, stream)
    sv.set_state(P.blast(n))
    import torch

    if warmup:
        sv.step(warmup, 0.7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv.step(steps, 0.7)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    B.mhd_timing(sv.h, True)
    t2 = time.perf_counter()
    sv.step(steps, 0.7)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    kern = {}
    for k, name in enumerate(B.KERNEL_KINDS):
        ms, cnt = B.mhd_timing_read(sv.h, k)
        kern[name] = (ms, cnt)
    B.mhd_timing(sv.h, False)
    reps = []
    for _ in range(repeats):
        ta = time.perf_counter()
        sv.step(steps, 0.7)
        torch.cuda.synchronize()
        reps.append(time.perf_counter() - ta)
    divb = sv.divb_max()
    t_sim, s_done = sv.time()
    sv.close()
    return (t1 - t0), kern, divb, t_sim, s_done, (t3 - t2), reps


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "blast256_traffic.txt")
# the kernels' source and the compiler flags they are built with
KERNEL_SOURCES = (os.path.join(HERE, "paper_0908_4362_amd", "csrc", "mhd_kernels_impl.h"),
                  os.path.join(HERE, "paper_0908_4362_amd", "build.py"))


def kernel_fingerprint():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(prec, kind, n):
    """HBM bytes per launch of one kernel kind from the committed counter summary, or None when the
    summary is for another workload or the kernel source has changed since the counters were taken."""
    if n != 256 or not os.path.exists(TRAFFIC_FILE):
        return None
    sha = kernel_fingerprint()
    table, src = {}, None
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            f = line.split()
            if not f or f[0].startswith("#"):
                continue
            if f[0] == "source_sha256":
                src = f[1]
            elif len(f) == 4:
                table[(f[0], f[1])] = int(f[2]) + int(f[3])
    if src != sha:
        return None
    return table.get((prec, kind))


def step_roofline(sec_per_step, ncell, esize):
    """The whole step against HBM: the path's minimum of STEP_WORDS words per cell (every directional
    operator reads and writes the 8-field state once, plus the CFL read) per step time, as a fraction
    of the 8 TB/s peak."""
    nbytes = STEP_WORDS * esize * ncell
    ach = nbytes / sec_per_step / 1e9
    return {"bound": "hbm", "words_per_cell": STEP_WORDS, "bytes_per_step": nbytes, "achieved": round(ach, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
            "ms_per_step_at_60pct": round(nbytes / (0.6 * HBM_PEAK_GBS * 1e9) * 1e3, 4)}


def roofline(kern, ncell, esize, n):
    total = {k: v[0] for k, v in kern.items() if v[1] > 0}
    dom = max(total, key=total.get)
    ms, cnt = kern[dom]
    avg_s = ms / cnt / 1e3
    bytes_per_launch = WORDS_PER_CELL[dom] * ncell * esize
    achieved = bytes_per_launch / avg_s / 1e9
    return dom, {
        "bound": "hbm",
        "kernel": dom,
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic("f64" if esize == 8 else "f32", dom, n),
        "avg_launch_ms": round(ms / cnt, 5),
        "bytes_per_launch": bytes_per_launch,
    }


def run_batched(B, P, count, steps, warmup, dtype, tune_reps):
    """The batched workload: every problem advanced `warmup` + `steps` full steps by one batch, then
    by its own plain solver; the timed regions are the `steps` steps of each."""
    import numpy as np
    import torch

    specs = P.alfven_batch_specs(count)
    npd = np.float64 if dtype == B.MHD_F64 else np.float32
    tdt = torch.float64 if dtype == B.MHD_F64 else torch.float32

    def state(sp):
        return P.alfven_111(sp["n"], sp["b0"], sp["amp"], sp["gamma"], dtype=npd)

    cells = sum(sp["n"] ** 3 for sp in specs)
    t0 = time.perf_counter()
    bt = B.Batch(dtype)
    ids = [bt.add(state(sp), sp["gamma"], B.MHD_BC_PERIODIC) for sp in specs]
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    if tune_reps:
        bt.autotune(tune_reps)
    tune_s = time.perf_counter() - t0
    bt.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.step(steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    print("bench: batched %d problems, %d cells: %.3f s for %d steps" % (count, cells, t_batch, steps),
          file=sys.stderr, flush=True)
    t_plain, same = 0.0, 0
    for sp, pid in zip(specs, ids):
        n = sp["n"]
        with B.Solver(n, n, n, sp["gamma"], B.MHD_BC_PERIODIC, dtype) as sv:
            sv.set_state(state(sp))
            sv.step(warmup)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sv.step(steps)
            torch.cuda.synchronize()
            t_plain += time.perf_counter() - t0
            a = torch.empty(8 * n ** 3, dtype=tdt, device="cuda")
            b = torch.empty_like(a)
            B.mhd_get_state_device(sv.h, a)
            B.mhd_batch_get_state_device(bt.b, pid, b)
            torch.cuda.synchronize()
            same += int(torch.equal(a, b))
    bt.close()
    return {
        "workload": "%d periodic linear Alfven waves, n^3 with n drawn from {32,48,64,96,128}, %s, CFL 0.7"
                    % (count, "FP64" if dtype == B.MHD_F64 else "FP32"),
        "problems": count,
        "cells": cells,
        "steps": steps,
        "warmup": warmup,
        "value": round(cells * steps / t_batch, 1),
        "unit": "cell-updates/s",
        "ms_per_step": round(t_batch * 1e3 / steps, 3),
        "plain_loop_value": round(cells * steps / t_plain, 1),
        "speedup_vs_plain_loop": round(t_plain / t_batch, 3),
        "identical_to_plain": same,
        "graphs": True,
        "autotune_reps": tune_reps,
        "setup_s": round(setup_s, 2),
        "autotune_s": round(tune_s, 2),
    }


class _Producer:
    """Builds request states in arrival order on a few host threads, a bounded
    number ahead of the consumer (numpy releases the GIL for the bulk work)."""

    def __init__(self, P, specs, ahead=16, workers=4):
        from collections import deque
        from concurrent.futures import ThreadPoolExecutor

        import numpy as np

        self.pool = ThreadPoolExecutor(max_workers=workers)
        self.specs = specs
        self.make = lambda sp: P.serving_state(sp, np.float64 if sp["dtype"] == 1 else np.float32)
        self.window = deque()
        self.k = 0
        for _ in range(min(ahead, len(specs))):
            self._push()

    def _push(self):
        if self.k < len(self.specs):
            self.window.append(self.pool.submit(self.make, self.specs[self.k]))
            self.k += 1

    def next(self):
        st = self.window.popleft().result()
        self._push()
        if not self.window:
            self.pool.shutdown(wait=False)
        return st


def _pct(xs, q):
    import numpy as np

    return round(float(np.percentile(np.asarray(xs), q)), 4)


def build_states(P, specs):
    """Every request's initial state, built on a few host threads before any timed run (a request
    arrives with its state). Vortex requests of one grid size and dtype have the same initial state,
    so they share one (read-only) array; each blast request has its own."""
    key = [("vortex", sp["n"], sp["dtype"]) if sp["kind"] == "vortex" else i for i, sp in enumerate(specs)]
    uniq = {}
    for i, k in enumerate(key):
        uniq.setdefault(k, i)
    order = sorted(uniq.values())
    prod = _Producer(P, [specs[i] for i in order])
    built = {i: prod.next() for i in order}
    return [built[uniq[k]] for k in key]


def serve_once(B, P, specs, arrivals, budget, max_cells=None, states=None):
    """Open-loop run: request i arrives, with its state already built, at arrivals[i] seconds after
    the start; returns (latencies, makespan, late submissions)."""
    n = len(specs)
    if states is None:
        states = build_states(P, specs)
    lat = [0.0] * n
    idx = {}
    late = 0
    with B.Server(budget, max_cells=max_cells) as srv:
        t0 = B.mhd_server_now()
        nxt = done = 0
        running = queued = 0
        last = t0
        while done < n:
            now = B.mhd_server_now() - t0
            while nxt < n and arrivals[nxt] <= now:
                sp = specs[nxt]
                st = states[nxt]
                if B.mhd_server_now() - t0 > arrivals[nxt] + 0.05:
                    late += 1
                # lent, not copied: the state stays alive in `states` for the whole run
                rid = srv.submit(st, sp["gamma"], B.MHD_BC_PERIODIC, sp["dtype"], sp["nsteps"], lend=True)
                idx[rid] = nxt
                nxt += 1
                now = B.mhd_server_now() - t0
            if nxt > done:     # submitted requests not yet finished (queued, running or to retire)
                running, queued = srv.tick()
            for rid in srv.finished():
                info = srv.info(rid)
                if info["status"] != B.MHD_OK:
                    raise RuntimeError("request %d failed with status %d" % (rid, info["status"]))
                i = idx.pop(rid)
                lat[i] = info["t_finish"] - (t0 + arrivals[i])
                last = max(last, info["t_finish"])
                srv.meta.pop(rid, None)
                B.mhd_server_take(srv.s, rid, _scratch(specs[i]))
                done += 1
                if done % 16 == 0 or done == n:
                    print("bench: served %d/%d (%.2f s)" % (done, n, B.mhd_server_now() - t0), file=sys.stderr,
                          flush=True)
            if nxt == done and nxt < n:
                wait = arrivals[nxt] - (B.mhd_server_now() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.005))
    return lat, last - t0, late


_scratch_bufs = {}


def _scratch(sp):
    import numpy as np

    key = (sp["n"], sp["dtype"])
    if key not in _scratch_bufs:
        _scratch_bufs[key] = np.empty((8, sp["n"], sp["n"], sp["n"]),
                                      dtype=np.float64 if sp["dtype"] == 1 else np.float32)
    return _scratch_bufs[key]


def run_serving(B, P, count, fracs, budget, steps, max_cells=None, sat_count=256):
    import numpy as np
    import torch

    specs = P.serving_specs(count, nsteps=steps)
    work = [sp["n"] ** 3 * sp["nsteps"] for sp in specs]
    t0 = time.perf_counter()
    states = build_states(P, specs)
    print("bench: serving, %d request states built in %.1f s" % (count, time.perf_counter() - t0), file=sys.stderr,
          flush=True)
    # plain solves one at a time, as a serial server would spend them (create, copy in, step, copy out,
    # release), on a stream of their own so that their steps replay from graphs. A solve's time depends
    # on its grid and dtype only (the kernels do the same work for any values), so each (n, dtype) class
    # is timed twice on one of its requests and the faster time stands for every request of the class.
    pstream = torch.cuda.Stream()
    first = {}
    for i, sp in enumerate(specs):
        first.setdefault((sp["n"], sp["dtype"]), i)
    svc, stp = {}, {}
    for key, i in sorted(first.items()):
        sp, st = specs[i], states[i]
        n = sp["n"]
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            with B.Solver(n, n, n, sp["gamma"], B.MHD_BC_PERIODIC, sp["dtype"]) as sv:
                B.mhd_set_stream(sv.h, pstream)
                sv.set_state(st)
                t1 = time.perf_counter()
                sv.step(sp["nsteps"], 0.7)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                sv.get_state()
            tt = (time.perf_counter() - t0, t2 - t1)
            best = tt if best is None or tt[0] < best[0] else best
        svc[key], stp[key] = best
    service = [svc[(sp["n"], sp["dtype"])] for sp in specs]
    stepping = [stp[(sp["n"], sp["dtype"])] for sp in specs]
    print("bench: serving, plain solves %.2f s (stepping %.2f s) for all %d requests" % (sum(service), sum(stepping),
          count), file=sys.stderr, flush=True)
    # saturation: the first sat_count requests all present at the start
    m = min(sat_count, count)
    lat0, span0, _ = serve_once(B, P, specs[:m], [0.0] * m, budget, max_cells, states[:m])
    sat = m / span0
    print("bench: serving, saturation %.2f requests/s (first %d requests)" % (sat, m), file=sys.stderr, flush=True)
    rng = np.random.Generator(np.random.PCG64(P.MASTER_SEED + 501))
    gaps = rng.exponential(1.0, size=count)
    points = []
    for f in fracs:
        lam = f * sat
        arr = list(np.cumsum(gaps / lam) - gaps[0] / lam)
        lat, span, late = serve_once(B, P, specs, arr, budget, max_cells, states)
        # the same arrivals served first come, first served by plain solves
        fin, slat = 0.0, []
        for a, sv in zip(arr, service):
            fin = max(a, fin) + sv
            slat.append(fin - a)
        points.append({"rate_frac": f, "rate_rps": round(lam, 3), "p50_s": _pct(lat, 50), "p99_s": _pct(lat, 99),
                       "makespan_s": round(span, 2), "cell_updates_per_s": round(sum(work) / span, 1),
                       "late_submissions": late, "plain_fcfs_p50_s": _pct(slat, 50),
                       "plain_fcfs_p99_s": _pct(slat, 99), "plain_fcfs_makespan_s": round(fin, 2)})
        print("bench: serving at %.2f x saturation: p50 %.3f s p99 %.3f s" % (f, points[-1]["p50_s"],
              points[-1]["p99_s"]), file=sys.stderr, flush=True)
    del states
    return {
        "workload": "%d requests: blast / extruded Orszag-Tang, n^3 with n in {32..192}, FP32/FP64, %d steps, "
                    "Poisson arrivals at %s x the saturation rate" % (count, steps, ", ".join("%g" % f for f in fracs)),
        "requests": count,
        "hbm_budget_bytes": budget,
        "max_running_cells": max_cells if max_cells is not None else 1 << 24,
        "cell_updates": sum(work),
        "saturation_requests": m,
        "saturation_rps": round(sat, 3),
        "saturation_cell_updates_per_s": round(sum(work[:m]) / span0, 1),
        "saturation_p50_s": _pct(lat0, 50),
        "saturation_p99_s": _pct(lat0, 99),
        "plain_serial_cell_updates_per_s": round(sum(work) / sum(service), 1),
        "plain_serial_stepping_only_cell_updates_per_s": round(sum(work) / sum(stepping), 1),
        "plain_service_s_per_class": {"%d^3 %s" % (k[0], "fp64" if k[1] == 1 else "fp32"): round(v, 4)
                                      for k, v in sorted(svc.items())},
        "speedup_vs_plain_serial": round(sum(service[:m]) / span0, 3),
        "points": points,
    }


# The paper's own timing workloads and its GTX 480 ms per full step (FP32, FP64): context for the
# same workloads run here, not a target (other hardware).
PAPER_CONFIGS = [
    ("Brio-Wu 1D, 4096 cells, outflow", "brio_wu", 4096, (4.31, 5.95)),
    ("Orszag-Tang 2D, 512^2, periodic", "orszag_tang", 512, (43.94, 56.26)),
    ("Orszag-Tang 2D, 1024^2, periodic", "orszag_tang", 1024, (96.43, 144.48)),
    ("3D blast, 128^3, periodic, B = (1,1,1)/sqrt3", "blast3", 128, (161.33, 276.40)),
]


def run_paper_configs(B, P, steps=20, warmup=3, only=None):
    """The paper's timing workloads (all, or the one at index `only`, which also reports per-kernel
    ms/step from an instrumented pass of as many steps)."""
    import torch

    out = []
    stream = torch.cuda.Stream()   # a stream of its own: steps replay from graphs
    for idx, (name, kind, n, paper_ms) in enumerate(PAPER_CONFIGS):
        if only is not None and idx != only:
            continue
        if kind == "brio_wu":
            s, gamma, bc = P.brio_wu(n), 2.0, B.MHD_BC_OUTFLOW
        elif kind == "orszag_tang":
            s, gamma, bc = P.orszag_tang(n), 5.0 / 3.0, B.MHD_BC_PERIODIC
        else:
            r = 1.0 / math.sqrt(3.0)
            s, gamma, bc = P.blast(n, bvec=(r, r, r)), 5.0 / 3.0, B.MHD_BC_PERIODIC
        nz, ny, nx = s.shape[1:]
        row = {"workload": name}
        for dtype, label, pms in ((B.MHD_F32, "fp32", paper_ms[0]), (B.MHD_F64, "fp64", paper_ms[1])):
            with B.Solver(nx, ny, nz, gamma, bc, dtype) as sv:
                B.mhd_set_stream(sv.h, stream)
                sv.set_state(s)
                sv.step(warmup, 0.7)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sv.step(steps, 0.7)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / steps
                kern = None
                if only is not None:
                    B.mhd_timing(sv.h, True)
                    sv.step(steps, 0.7)
                    torch.cuda.synchronize()
                    kern = {k: round(B.mhd_timing_read(sv.h, i)[0] / steps, 4) for i, k in enumerate(B.KERNEL_KINDS)}
                    B.mhd_timing(sv.h, False)
            row[label] = {"ms_per_step": round(ms, 4), "cell_updates_per_s": round(nx * ny * nz / ms * 1e3, 1),
                          "paper_gtx480_ms_per_step": pms, "speedup_vs_paper": round(pms / ms, 1)}
            if kern is not None:
                row[label]["kernels_ms_per_step"] = kern
        out.append(row)
    return out


def host_cpus():
    """CPUs this process may run on (the box's share, whatever nproc shows)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        avail = min(avail, int(env))
    return max(1, avail)


def cpu_baseline(P, n, sample):
    """The oracle on the host cores: the OpenMP build on every available core
    for 1 warm-up + 2 timed full steps of the n^3 blast itself (the value),
    and the serial build pinned to one core for up to 3 steps of a sample^3
    box cut from the centre of the same blast (outflow edges)."""
    import numpy as np

    import oracle

    oracle.build()
    s = P.blast(n)
    threads = host_cpus()
    g = oracle.Grid(n, n, n, 5.0 / 3.0, oracle.PERIODIC)
    used = oracle.set_threads(threads)
    st, t, k = oracle.run(g, s, 1, 0.7)
    t0 = time.perf_counter()
    st, t, k = oracle.run(g, st, 2, 0.7, t, k)
    par = time.perf_counter() - t0
    oracle.set_threads(1)
    del st
    lo = (n - sample) // 2
    box = np.ascontiguousarray(s[:, lo:lo + sample, lo:lo + sample, lo:lo + sample])
    del s
    gb = oracle.Grid(sample, sample, sample, 5.0 / 3.0, oracle.OUTFLOW)
    try:
        old_aff = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {min(old_aff)})
    except (AttributeError, OSError):
        old_aff = None
    t0 = time.perf_counter()
    steps = 0
    while True:
        box, _, _ = oracle.run(gb, box, 1, 0.7, 0.0, steps)
        steps += 1
        if time.perf_counter() - t0 > 8.0 or steps >= 3:
            break
    ser = time.perf_counter() - t0
    if old_aff is not None:
        os.sched_setaffinity(0, old_aff)
    return {
        "value": round(n ** 3 * 2 / par, 1),
        "unit": "cell-updates/s",
        "cores": used,
        "kind": "oracle",
        "sample": "1 warm-up + 2 timed full steps of the %d^3 blast (periodic), FP64 C oracle built with OpenMP "
                  "(-O3, no FMA contraction; pencils of each sweep shared among %d threads, bitwise the serial "
                  "build)" % (n, used),
        "seconds_per_step": round(par / 2, 3),
        "serial": {"value": round(sample ** 3 * steps / ser, 1), "cores": 1,
                   "sample": "%d full step(s) of a %d^3 box cut from the centre of the %d^3 blast (outflow edges), "
                             "serial build pinned to one core" % (steps, sample, n)},
        "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count(), "available_cpus": threads},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=5,
                    help="further passes of K timed steps after the headline pass; their median is reported")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per axis (workload: 256)")
    ap.add_argument("--cpu-sample", type=int, default=96, help="edge of the box timed on the CPU oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=50)
    ap.add_argument("--batch-tune", type=int, default=3, help="autotuner launches per candidate (0: off)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving workload")
    ap.add_argument("--no-paper-configs", action="store_true", help="skip the paper's own timing workloads")
    ap.add_argument("--paper-only", type=int, default=None, choices=range(len(PAPER_CONFIGS)),
                    help="run only this one of the paper's timing workloads (0 Brio-Wu 4096, 1 Orszag-Tang 512^2, "
                         "2 Orszag-Tang 1024^2, 3 blast 128^3), with per-kernel times, and print its JSON line")
    ap.add_argument("--serve-count", type=int, default=1024)
    ap.add_argument("--serve-rates", default="0.75,1.0,1.25", help="arrival rates as fractions of saturation")
    ap.add_argument("--serve-sat-count", type=int, default=256,
                    help="requests of the closed-loop run that measures the saturation rate")
    ap.add_argument("--serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--serve-steps", type=int, default=100)
    ap.add_argument("--serve-max-cells", type=int, default=None,
                    help="server admission cap on running cells (default: the library's, 2^24; 0: none)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU; --gpus %d is not supported (a multi-GPU run would need a "
              "halo exchange per sub-operation and an all-reduce of c_max, which are not implemented)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch

    from paper_0908_4362_amd import binding as B
    from paper_0908_4362_amd import problems as P

    torch.cuda.set_device(0)
    if args.paper_only is not None:
        print("bench: paper timing workload %d only" % args.paper_only, file=sys.stderr, flush=True)
        print(json.dumps(run_paper_configs(B, P, args.steps, args.warmup, only=args.paper_only)[0]), flush=True)
        return
    stream = torch.cuda.Stream()   # a stream of its own (default priority): full steps replay from graphs
    n = args.n
    ncell = n ** 3
    if args.copy_calibration_mib:
        nbytes = args.copy_calibration_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print("bench: copy calibration %d bytes read + %d bytes written" % (nbytes, nbytes), file=sys.stderr,
              flush=True)
        del src, dst
    print("bench: %d^3 blast, fp64, %d warm-up + %d timed steps" % (n, args.warmup, args.steps), file=sys.stderr,
          flush=True)
    sec64, kern64, divb64, tsim, sdone, inst64, reps64 = run_gpu(B, P, n, B.MHD_F64, args.warmup, args.steps,
                                                                 stream, args.repeats)
    dom, roof = roofline(kern64, ncell, 8, n)
    out = {
        "metric": "cell-updates/s per full step",
        "value": round(ncell * args.steps / sec64, 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec64 * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "3D MHD blast wave, periodic %d^3, FP64, CFL 0.7" % n, "cells": ncell,
                   "global_batch": 1, "parallelism": "single GPU"},
        "roofline": roof,
        "effective_step_bandwidth_GBs": round(STEP_WORDS * 8 * ncell * args.steps / sec64 / 1e9, 1),
        "step_roofline": step_roofline(sec64 / args.steps, ncell, 8),
        "step_words": {"minimum": STEP_WORDS, "this_design": design_step_words(kern64, args.steps),
                       "cfl_fused_into_last_sweep": True},
        "kernels_ms_per_step": {k: round(v[0] / max(1, args.steps), 4) for k, v in kern64.items()},
        "instrumented_ms_per_step": round(inst64 * 1e3 / args.steps, 4),
        "repeats": repeat_summary(reps64, args.steps),
        "divb_max_after": divb64,
    }
    if not args.no_fp32:
        print("bench: %d^3 blast, fp32" % n, file=sys.stderr, flush=True)
        sec32, kern32, divb32, _, _, inst32, reps32 = run_gpu(B, P, n, B.MHD_F32, args.warmup, args.steps,
                                                              stream, args.repeats)
        _, roof32 = roofline(kern32, ncell, 4, n)
        out["fp32"] = {
            "value": round(ncell * args.steps / sec32, 1),
            "ms_per_step": round(sec32 * 1e3 / args.steps, 4),
            "roofline": roof32,
            "effective_step_bandwidth_GBs": round(STEP_WORDS * 4 * ncell * args.steps / sec32 / 1e9, 1),
            "step_roofline": step_roofline(sec32 / args.steps, ncell, 4),
            "kernels_ms_per_step": {k: round(v[0] / max(1, args.steps), 4) for k, v in kern32.items()},
            "instrumented_ms_per_step": round(inst32 * 1e3 / args.steps, 4),
            "repeats": repeat_summary(reps32, args.steps),
        }
    if not args.no_paper_configs:
        print("bench: the paper's timing workloads", file=sys.stderr, flush=True)
        out["paper_configs"] = run_paper_configs(B, P)
    if not args.no_batch:
        print("bench: batched workload", file=sys.stderr, flush=True)
        out["batched"] = run_batched(B, P, args.batch_count, args.batch_steps, 2, B.MHD_F32, args.batch_tune)
    if not args.no_serve:
        print("bench: serving workload", file=sys.stderr, flush=True)
        out["serving"] = run_serving(B, P, args.serve_count, [float(x) for x in args.serve_rates.split(",")],
                                     int(args.serve_budget_gb * (1 << 30)), args.serve_steps, args.serve_max_cells,
                                     args.serve_sat_count)
    if rank == 0 and not args.no_cpu_baseline:
        print("bench: cpu oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(P, n, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

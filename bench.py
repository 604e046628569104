#!/usr/bin/env python3
"""Benchmark of the MHD time step on one MI355X.

Workload: the 3D MHD blast wave on a periodic 256^3 unit cube (gamma = 5/3,
rho = 1, p = 10 inside r < 0.1 about the centre and 0.1 outside, uniform
B = (1/sqrt2, 1/sqrt2, 0), v = 0), CFL 0.7, W warm-up steps then K timed full
steps. A full step is the CFL reduction plus the forward and reverse sweeps
(12 directional sub-operations) and advances t by 2 dt. The state is resident
in HBM before the timed region; the whole step runs in the HIP library.

Prints one JSON line: cell-updates/s per full step (FP64 headline, FP32 next
to it), the roofline of the dominant kernel from HIP events recorded on the
handle's stream during the timed region, and the CPU oracle timed on a bounded
sample of the same workload.
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
WORDS_PER_CELL = {"cfl": 8, "fluid_x": 13, "fluid_y": 13, "fluid_z": 13, "ct_x": 8, "ct_y": 8, "ct_z": 8}
STEP_WORDS = 104  # minimum per full step: 6 directional operators x (8 read + 8 written) + 8 for the CFL


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def run_gpu(B, P, n, dtype, warmup, steps, stream):
    nx = ny = nz = n
    sv = B.Solver(nx, ny, nz, 5.0 / 3.0, B.MHD_BC_PERIODIC, dtype)
    B.mhd_set_stream(sv.h, stream)
    sv.set_state(P.blast(n))
    import torch

    if warmup:
        sv.step(warmup, 0.7)
    torch.cuda.synchronize()
    B.mhd_timing(sv.h, True)
    t0 = time.perf_counter()
    sv.step(steps, 0.7)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = {}
    for k, name in enumerate(B.KERNEL_KINDS):
        ms, cnt = B.mhd_timing_read(sv.h, k)
        kern[name] = (ms, cnt)
    B.mhd_timing(sv.h, False)
    divb = sv.divb_max()
    t_sim, s_done = sv.time()
    sv.close()
    return (t1 - t0), kern, divb, t_sim, s_done


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "blast256_traffic.txt")
KERNEL_SOURCE = os.path.join(HERE, "paper_0908_4362_amd", "csrc", "mhd_kernels_impl.h")


def measured_traffic(prec, kind, n):
    """HBM bytes per launch of one kernel kind from the committed counter summary, or None when the
    summary is for another workload or the kernel source has changed since the counters were taken."""
    if n != 256 or not os.path.exists(TRAFFIC_FILE):
        return None
    with open(KERNEL_SOURCE, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()[:16]
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


def cpu_baseline(P, n, sample):
    """The oracle, single thread, on a bounded sample: one full step of a
    sample^3 box cut from the centre of the n^3 blast (outflow edges)."""
    import numpy as np

    import oracle

    s = P.blast(n)
    lo = (n - sample) // 2
    box = np.ascontiguousarray(s[:, lo:lo + sample, lo:lo + sample, lo:lo + sample])
    g = oracle.Grid(sample, sample, sample, 5.0 / 3.0, oracle.OUTFLOW)
    oracle.build()
    t0 = time.perf_counter()
    steps = 0
    while True:
        box, _, _ = oracle.run(g, box, 1, 0.7, 0.0, steps)
        steps += 1
        if time.perf_counter() - t0 > 8.0 or steps >= 3:
            break
    dt = time.perf_counter() - t0
    return {
        "value": round(sample ** 3 * steps / dt, 1),
        "unit": "cell-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "%d full step(s) of a %d^3 box cut from the centre of the %d^3 blast, serial FP64 C oracle, "
                  "host CPU: %s" % (steps, sample, n, cpu_model()),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256, help="cells per axis (workload: 256)")
    ap.add_argument("--cpu-sample", type=int, default=96, help="edge of the box timed on the CPU oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
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
    stream = torch.cuda.current_stream()
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
    sec64, kern64, divb64, tsim, sdone = run_gpu(B, P, n, B.MHD_F64, args.warmup, args.steps, stream)
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
        "kernels_ms_per_step": {k: round(v[0] / max(1, args.steps), 4) for k, v in kern64.items()},
        "divb_max_after": divb64,
    }
    if not args.no_fp32:
        print("bench: %d^3 blast, fp32" % n, file=sys.stderr, flush=True)
        sec32, kern32, divb32, _, _ = run_gpu(B, P, n, B.MHD_F32, args.warmup, args.steps, stream)
        _, roof32 = roofline(kern32, ncell, 4, n)
        out["fp32"] = {
            "value": round(ncell * args.steps / sec32, 1),
            "ms_per_step": round(sec32 * 1e3 / args.steps, 4),
            "roofline": roof32,
            "effective_step_bandwidth_GBs": round(STEP_WORDS * 4 * ncell * args.steps / sec32 / 1e9, 1),
            "kernels_ms_per_step": {k: round(v[0] / max(1, args.steps), 4) for k, v in kern32.items()},
        }
    if rank == 0 and not args.no_cpu_baseline:
        print("bench: cpu oracle sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(P, n, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

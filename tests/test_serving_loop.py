"""CPU check of the open-loop serving driver in bench.py against a Python
model of the request server's tick semantics (admission under a budget in
arrival order, one step per tick, retirement on the tick after the last
step): every request is served, latencies are non-negative, and a burst
where every request arrives at once (all queued before the first tick)
terminates."""
from __future__ import annotations

import collections
import time
import types

import numpy as np

import bench
from paper_0908_4362_amd import problems as P


class ModelServer:
    def __init__(self, budget, cfl=0.7, max_cells=None):
        self.budget, self.used = budget, 0
        self.max_cells = (1 << 24) if max_cells is None else max_cells
        self.reqs, self.queue, self.running, self.done = {}, collections.deque(), [], collections.deque()
        self.next_id, self.meta, self.s, self.ticks, self.peak = 1, {}, self, 0, 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        pass

    def submit(self, st, gamma, bc, dtype, nsteps, lend=False):
        n = st.shape[1]
        b = 16 * n ** 3 * (8 if dtype else 4)
        assert b <= self.budget
        rid = self.next_id
        self.next_id += 1
        self.reqs[rid] = {"bytes": b, "cells": n ** 3, "nsteps": nsteps, "issued": 0, "t_submit": time.monotonic(), "t_admit": -1.0,
                          "t_finish": -1.0, "status": 0}
        self.queue.append(rid)
        self.meta[rid] = (st.shape, dtype)
        return rid

    def tick(self):
        self.ticks += 1
        keep = []
        for rid in self.running:
            r = self.reqs[rid]
            if r["issued"] >= r["nsteps"]:
                self.used -= r["bytes"]
                r["t_finish"] = time.monotonic()
                self.done.append(rid)
            else:
                keep.append(rid)
        self.running = keep
        cells = sum(self.reqs[rid]["cells"] for rid in self.running)
        while self.queue:
            r = self.reqs[self.queue[0]]
            if self.used + r["bytes"] > self.budget:
                break
            if self.max_cells and self.running and cells + r["cells"] > self.max_cells:
                break
            cells += r["cells"]
            self.used += r["bytes"]
            r["t_admit"] = time.monotonic()
            self.running.append(self.queue.popleft())
        self.peak = max(self.peak, self.used)
        for rid in self.running:
            self.reqs[rid]["issued"] += 1
        return len(self.running), len(self.queue)

    def finished(self):
        out = list(self.done)
        self.done.clear()
        return out

    def info(self, rid):
        return dict(self.reqs[rid])


def model_binding(servers):
    def make(budget, cfl=0.7, max_cells=None):
        s = ModelServer(budget, cfl, max_cells)
        servers.append(s)
        return s

    return types.SimpleNamespace(Server=make, mhd_server_now=time.monotonic, MHD_OK=0, MHD_BC_PERIODIC=0,
                                 mhd_server_take=lambda s, rid, out: s.reqs.pop(rid))


def test_burst_arrivals_are_all_served():
    servers = []
    specs = P.serving_specs(24, nsteps=5, sizes=(8, 12, 16))
    budget = 6 * 16 * 16 ** 3 * 8
    lat, span, late = bench.serve_once(model_binding(servers), P, specs, [0.0] * len(specs), budget)
    assert len(lat) == len(specs) and min(lat) >= 0.0 and span > 0.0
    assert servers[0].peak <= budget and not servers[0].reqs


def test_spread_arrivals_are_all_served():
    servers = []
    specs = P.serving_specs(16, nsteps=3, sizes=(8, 12))
    arr = list(np.cumsum(np.full(len(specs), 0.003)))
    lat, span, late = bench.serve_once(model_binding(servers), P, specs, arr, 1 << 30)
    assert min(lat) >= 0.0 and span >= arr[-1]
    assert not servers[0].reqs


def test_burst_under_a_cell_cap_is_served_in_order():
    """The bench loop with the server's admission cell cap: every request is
    served even when the cap holds the queue back, including a cap below a
    single request (it then runs alone)."""
    for cap in (1, 2 * 12 ** 3, 0):
        servers = []
        specs = P.serving_specs(12, nsteps=3, sizes=(8, 12, 16))
        lat, span, late = bench.serve_once(model_binding(servers), P, specs, [0.0] * len(specs), 1 << 30,
                                           max_cells=cap)
        assert len(lat) == len(specs) and min(lat) >= 0.0
        assert not servers[0].reqs and servers[0].max_cells == cap

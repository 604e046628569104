"""Writes tests/golden/oracle_snapshot.json from the oracle only (small cases:
a few steps of Brio-Wu, Orszag-Tang and a random smooth 3D state). Run from the
repository root: python -m tests.golden.make_snapshot"""
from __future__ import annotations

import json
import os

import numpy as np

from paper_0908_4362_amd import problems as P

CASES = ("brio_wu_32_outflow_5", "orszag_tang_16_3", "random_smooth_6x5x4_2")


def build_case(orc, name):
    if name == "brio_wu_32_outflow_5":
        g = orc.Grid(32, 1, 1, 2.0, orc.OUTFLOW)
        out, _, _ = orc.run(g, P.brio_wu(32), 5, 0.7)
        return out[[0, 1, 4, 6]].ravel()
    if name == "orszag_tang_16_3":
        g = orc.Grid(16, 16, 1, 5.0 / 3.0)
        out, _, _ = orc.run(g, P.orszag_tang(16), 3, 0.7)
        return out[:, 0, ::3, ::3].ravel()
    if name == "random_smooth_6x5x4_2":
        g = orc.Grid(6, 5, 4, 5.0 / 3.0)
        out, _, _ = orc.run(g, P.random_smooth(6, 5, 4, seed=P.MASTER_SEED), 2, 0.7)
        return out[:, ::2, ::2, ::2].ravel()
    raise KeyError(name)


def main():
    import oracle

    cases = [{"name": n, "values": [float(v) for v in build_case(oracle, n)]} for n in CASES]
    path = os.path.join(os.path.dirname(__file__), "oracle_snapshot.json")
    with open(path, "w") as fh:
        json.dump({"_writer": "tests/golden/make_snapshot.py (oracle only)", "cases": cases}, fh)
    print("wrote", path)


if __name__ == "__main__":
    main()

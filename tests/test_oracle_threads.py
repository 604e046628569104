"""The OpenMP build of the oracle (the same source with the pencils of each
sweep shared among threads) gives the serial build's bits: full steps,
single sweeps, c_max and div B, under both boundary conditions, on grids with
uneven pencil counts."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_0908_4362_amd import problems as P


@pytest.fixture
def threads():
    yield
    oracle.set_threads(1)


@pytest.mark.parametrize("bc", [oracle.PERIODIC, oracle.OUTFLOW])
def test_threaded_oracle_equals_serial(threads, bc):
    nx, ny, nz = 21, 17, 13
    s = P.random_smooth(nx, ny, nz, seed=P.MASTER_SEED + 700 + bc)
    g = oracle.Grid(nx, ny, nz, 5.0 / 3.0, bc)
    res = {}
    for n in (1, 4):
        used = oracle.set_threads(n)
        assert used == n
        st, t, k = oracle.run(g, s, 3, 0.7)
        sweeps = [oracle.fluid_sweep(g, s, d, 0.05) for d in range(3)] + [oracle.ct_sweep(g, s, d, 0.05)
                                                                          for d in range(3)]
        res[n] = (st, t, k, sweeps, oracle.cmax(g, s), oracle.divb_max(g, st + 1e-3 * (np.arange(st.size) % 7
                                                                                      ).reshape(st.shape)))
    a, b = res[1], res[4]
    assert np.array_equal(a[0], b[0]) and a[1] == b[1] and a[2] == b[2]
    for x, y in zip(a[3], b[3]):
        assert np.array_equal(x, y)
    assert a[4] == b[4] and a[5] == b[5]


def test_threaded_cmax_propagates_nan(threads):
    s = P.random_smooth(8, 8, 8, seed=P.MASTER_SEED + 702)
    s[0, 5, 6, 7] = np.nan
    g = oracle.Grid(8, 8, 8, 5.0 / 3.0)
    oracle.set_threads(3)
    assert np.isnan(oracle.cmax(g, s))

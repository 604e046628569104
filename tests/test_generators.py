"""CPU checks of the seeded input generators of the batched workload."""
from __future__ import annotations

import math

import numpy as np

from paper_0908_4362_amd import problems as P


def test_alfven_batch_specs_follow_the_recipe():
    specs = P.alfven_batch_specs(200)
    assert specs == P.alfven_batch_specs(200)          # seeded
    assert specs != P.alfven_batch_specs(200, seed=1)
    khat = np.ones(3) / math.sqrt(3.0)
    sizes = set()
    for sp in specs:
        b = np.asarray(sp["b0"])
        assert abs(np.linalg.norm(b) - 1.0) < 1e-12
        assert abs(khat @ b) >= 0.1 and np.linalg.norm(np.cross(khat, b)) >= 0.1
        assert 1e-4 <= sp["amp"] <= 1e-2
        sizes.add(sp["n"])
    assert sizes == set(P.BATCH_SIZES)


def test_alfven_111_is_the_linear_wave_state():
    for n, sp in zip((8, 12, 17), P.alfven_batch_specs(3, seed=5)):
        b0 = np.asarray(sp["b0"])
        amp = 0.01
        khat = np.ones(3) / math.sqrt(3.0)
        nd = np.cross(khat, b0)
        nd /= np.linalg.norm(nd)
        sg = 1.0 if khat @ b0 >= 0 else -1.0
        ref = P.linear_wave(n, n, n, (1, 1, 1), 1.0, 0.6, (0, 0, 0), tuple(b0), 5.0 / 3.0,
                            dv=tuple(-sg * amp * nd), db=amp, db_dir=tuple(nd))
        got = P.alfven_111(n, b0, amp)
        assert np.abs(got - ref).max() <= 1e-13


def test_alfven_111_field_is_divergence_free_and_eigenvector():
    sp = P.alfven_batch_specs(1, seed=9)[0]
    n = 20
    s = P.alfven_111(n, sp["b0"], 1e-3)
    bx, by, bz = s[5], s[6], s[7]
    div = (np.roll(bx, -1, axis=2) - bx) + (np.roll(by, -1, axis=1) - by) + (np.roll(bz, -1, axis=0) - bz)
    assert np.abs(div).max() <= 1e-14
    # Alfven eigenvector: dv = -sign(k.b0) dB / sqrt(rho), both along k x b0
    khat = np.ones(3) / math.sqrt(3.0)
    b0 = np.asarray(sp["b0"])
    v = s[1:4, 3, 2, 1]
    db = np.array([0.5 * (s[5, 3, 2, 1] + s[5, 3, 2, 2]), 0.5 * (s[6, 3, 2, 1] + s[6, 3, 3, 1]),
                   0.5 * (s[7, 3, 2, 1] + s[7, 4, 2, 1])]) - b0
    sg = 1.0 if khat @ b0 >= 0 else -1.0
    # the face field of the discrete curl differs from the centred wave by O((k h)^2)
    kh = 2.0 * math.pi / n
    assert np.linalg.norm(v + sg * db) <= kh * kh * np.linalg.norm(v)
    assert abs(v @ khat) <= 1e-15 and abs(v @ b0) <= 1e-15


def test_serving_specs_follow_the_recipe():
    specs = P.serving_specs(400)
    assert specs == P.serving_specs(400)
    kinds = [sp["kind"] for sp in specs]
    assert 150 < kinds.count("blast") < 250
    assert 150 < sum(sp["dtype"] for sp in specs) < 250
    assert set(sp["n"] for sp in specs) == set(P.SERVE_SIZES)
    for sp in specs:
        assert sp["nsteps"] == 100
        if sp["kind"] == "blast":
            assert 1.0 <= sp["p_in"] <= 100.0 and 0.05 <= sp["radius"] <= 0.15
            assert np.linalg.norm(sp["bvec"]) <= 1.0


def test_serving_state_equals_the_paper_problem_generators():
    for sp in P.serving_specs(12, seed=3, sizes=(8, 12, 20)):
        n = sp["n"]
        if sp["kind"] == "blast":
            ref = P.blast(n, p_in=sp["p_in"], p_out=0.1, radius=sp["radius"], bvec=sp["bvec"])
        else:
            ref = P.orszag_tang(n, nz=n)
        assert np.array_equal(P.serving_state(sp), ref)
        assert np.array_equal(P.serving_state(sp, np.float32), ref.astype(np.float32))

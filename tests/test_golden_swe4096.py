"""The stored 1000-step oracle states of the 4096^2 reflective workload
(tests/golden/swe4096_1000steps.json, written by make_swe4096_1000.py from
oracle/ alone): every run conserves the initial mass (reflective walls), the
transverse scheme gives the same state from the FP64 initial state and from
its FP32 rounding (a stable scheme keeps a 1e-8 perturbation small), and the
paper's scheme does not (its weak 2-D instability amplifies the rounding
perturbation over 1000 steps into visible waves)."""
import json
import math
import os

import numpy as np
import pytest

from paper_1107_2157_amd import ics

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "swe4096_1000steps.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)


def runs(gold, scheme):
    return {r["start"]: r for r in gold["runs"] if r["scheme"] == scheme}


def test_every_run_conserves_the_initial_mass(gold):
    h, _, _ = ics.bumps_state(4096, 4096, seed=2, periodic=False, count=8)
    h = h.numpy()
    m0 = {"f64": math.fsum(h.ravel()), "f32": math.fsum(h.astype(np.float32).astype(np.float64).ravel())}
    assert gold["steps"] == 1000 and len(gold["runs"]) == 4
    for r in gold["runs"]:
        assert r["finite"]
        assert abs(r["fields"]["h"]["sum"] - m0[r["start"]]) <= 1e-12 * m0[r["start"]], (r["scheme"], r["start"])


def test_transverse_is_insensitive_to_the_fp32_rounding(gold):
    r = runs(gold, "transverse")
    assert abs(r["f64"]["t"] - r["f32"]["t"]) <= 1e-6 * r["f64"]["t"]
    for k in ("h", "hu", "hv"):
        a, b = np.array(r["f64"]["fields"][k]["lattice"]), np.array(r["f32"]["fields"][k]["lattice"])
        assert np.max(np.abs(a - b)) <= 1e-5


def test_paper_scheme_amplifies_the_fp32_rounding(gold):
    r = runs(gold, "paper")
    a, b = np.array(r["f64"]["fields"]["h"]["lattice"]), np.array(r["f32"]["fields"]["h"]["lattice"])
    assert np.max(np.abs(a - b)) > 1e-3
    assert r["f32"]["fields"]["hu"]["max_abs"] > 2 * r["f64"]["fields"]["hu"]["max_abs"]

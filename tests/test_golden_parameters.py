"""The paper's printed model parameters and scenario values (tests/golden/paper_parameters.json,
each entry with its citation) against the ones the workloads, tests and benchmarks use."""
import json
import math
import os

import pytest

from paper_1903_07715_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_parameters.json")))


def test_running_example_defaults():
    g = GOLD["running_example"]
    d = W.double_integrator()
    assert d.id == W.DYN_DOUBLE_INTEGRATOR
    assert d.params == (g["ubar"], g["b"], g["dbar"])


def test_quad10_dynamics_parameters():
    q = GOLD["quad10"]
    g, d0, d1, n0, smax, dbar = W.quad10_xy().params
    assert (d0, d1, n0) == (q["d0"], q["d1"], q["n0"])
    assert smax == pytest.approx(math.radians(q["S_max_degrees"]), rel=1e-15)
    assert dbar == q["base"]["dbar_xy"]
    gz, kt, m, tmin, tmax, dz = W.quad10_z().params
    assert gz == g and kt == q["kT"] and m == q["base"]["m"] and dz == q["base"]["dbar_z"]
    assert tmin == q["T_min"] and tmax == pytest.approx(q["T_max_over_g"] * g, rel=1e-15)


def test_quad10_scenarios():
    q = GOLD["quad10"]
    for tag in ("base", "heavier", "lighter"):
        assert W.QUAD10_SCENARIOS[tag] == (q[tag]["m"], q[tag]["dbar_xy"])
    probs = W.quad10_problems(*W.QUAD10_SCENARIOS["heavier"], n_xy=7, n_z=7)
    assert probs[0].dyn.params[5] == q["heavier"]["dbar_xy"] and probs[2].dyn.params[2] == q["heavier"]["m"]


def test_table1_discount_factor():
    assert W.TABLE1_DISCOUNT == GOLD["discounted_reachability"]["factor"]

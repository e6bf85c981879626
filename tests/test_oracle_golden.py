"""Oracle regression against stored values written by tests/golden/make_golden.py (oracle only),
and the paper's parameter block (tests/golden/paper_parameters.json, each value cited)."""
import json
import os

import numpy as np

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_water_golden(water, water_oracle):
    g = json.load(open(os.path.join(GOLD, "water_tiny.json")))
    om = water_oracle
    sol = O.full_solution(om, water.P)
    assert om.M == g["M"] and om.nbf == g["nbf"]
    assert om.keep_idx[:20].tolist() == g["keep_idx_head"]
    assert om.pairs()["a"].shape[0] == g["n_pairs_fock"]
    assert abs(sol["E"] - g["E"]) <= 1e-12 * abs(g["E"])
    assert np.allclose(sol["c"][:8], g["c_head"], rtol=1e-12, atol=0)
    assert np.allclose(sol["q"][:8], g["q_head"], rtol=1e-10, atol=0)


def test_paper_parameters_fixture():
    p = json.load(open(os.path.join(GOLD, "paper_parameters.json")))
    assert p["eps"]["value"] == 78.39 and p["schwarz_thresh"]["value"] == 1e-12
    # Eq. 21 as used in Sec. 4b-i with the stored constants
    e = 1e-4
    d = O.dynamic_threshold(e)
    assert abs(p["dynamic_err_coef"]["value"] * d ** p["dynamic_err_power"]["value"]
               - p["dynamic_safety"]["value"] * e) < 1e-18

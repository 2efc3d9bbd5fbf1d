"""The oracle reproduces its stored regression fixture (tests/golden)."""
import json
import os

import numpy as np

import oracle
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_config0_fixture_unchanged():
    with open(os.path.join(HERE, "golden", "config0_oracle.json")) as f:
        gold = json.load(f)
    w = W.config0()
    e_min, e_max, a, b = oracle.workload_bounds(w)
    assert abs(a - gold["bounds"]["a"]) == 0.0 and b == gold["bounds"]["b"]
    mu_ee, mu_he = oracle.workload_moments(w, a, b)
    rows = gold["rows"]
    assert np.max(np.abs(mu_ee[rows] - np.array(gold["mu_ee"]))) < 1e-14
    assert np.max(np.abs(mu_he[rows] - np.array(gold["mu_he"]))) < 1e-14
    new = oracle.gap_map(mu_he, w.U).real
    assert np.max(np.abs(new - np.array(gold["delta_one_step"]))) < 1e-14
    ld = oracle.ldos(mu_ee[rows], np.array(gold["ldos_energies"]), a, b)
    assert np.max(np.abs(ld - np.array(gold["ldos"]))) < 1e-13

"""Writes the stored oracle fixtures in this folder.  Calls only ``oracle`` and
``workloads``; run from the repository root:  python tests/golden/make_golden.py

The paper prints no numerical results (its two figures carry no data), so the
fixtures here are oracle regression values for the 16x16 workload with one
impurity (V = 5 at the centre), kept so that any later change to the oracle's
arithmetic shows up as a diff; their correctness rests on the pins in
tests/test_oracle_pins.py (exact diagonalisation, closed forms, invariants).
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    w = W.config0()
    e_min, e_max, a, b = oracle.workload_bounds(w)
    mu_ee, mu_he = oracle.workload_moments(w, a, b)
    new = oracle.gap_map(mu_he, w.U).real
    rows = [0, 17, 136, 255]
    E = [-1.0, -0.1, 0.0, 0.05, 0.7]
    out = {
        "workload": w.name,
        "bounds": {"E_min": e_min, "E_max": e_max, "a": a, "b": b},
        "rows": rows,
        "mu_ee": mu_ee[rows].tolist(),
        "mu_he": mu_he[rows].tolist(),
        "delta_one_step": new.tolist(),
        "ldos_energies": E,
        "ldos": oracle.ldos(mu_ee[rows], np.array(E), a, b).tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config0_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()

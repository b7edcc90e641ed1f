"""Consistency of the stored oracle run of the large workload
(tests/golden/config3_cycles.json, written by make_config3_reference.py from
the oracle alone): Parseval for the stored density (sum = p), ascending Ritz
values that rise from cycle to cycle (Rayleigh-Ritz values of a filtered
subspace are upper bounds that decrease towards the spectrum: each cycle's
lowest value is <= the previous one), p at the largest gap of its window, and
residuals that shrink from cycle to cycle."""
import json
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config3_cycles.json")


def test_stored_oracle_run_is_consistent():
    d = json.load(open(GOLD))
    assert d["npw"] == 115313 and d["nband"] == 2048 and d["degree"] == 12
    assert len(d["cycles"]) == 4
    p = d["p"]
    assert abs(d["rho_sum"] - p) <= 1e-9 * p
    assert max(d["rho_values"]) <= d["rho_max"] and min(d["rho_values"]) >= 0.0
    evs = [np.array(c["eval"]) for c in d["cycles"]]
    for ev in evs:
        assert np.all(np.diff(ev) >= 0.0)
    for prev, cur in zip(evs, evs[1:]):
        assert cur[0] <= prev[0] + 1e-12
    gaps = np.diff(evs[-1][999:1048])
    assert abs(d["gap_at_p"] - gaps.max()) <= 1e-15 and 1000 <= p <= 1048
    assert evs[-1][p] - evs[-1][p - 1] == d["gap_at_p"]
    res = [c["max_residual"] for c in d["cycles"]]
    assert all(b < a for a, b in zip(res, res[1:]))
    assert abs(max(d["last_residuals"]) - res[-1]) <= 1e-15

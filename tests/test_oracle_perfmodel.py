"""The oracle's performance model against the paper's two tables of
right-hand-side counts (section "Performance Model", Tables t:perfmodelthird
and t:perfmodelfourth), from the paper's grid sizes (section "Guiding
Experiment") and stable-step ratios r_RK4 (Tables t:thirdstab, t:fourthstab),
with t = dt_RK4 as the paper takes it."""
import json
import os

import numpy as np
import pytest

from oracle import perfmodel

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def test_grid_sizes_are_the_guiding_experiment_grids():
    g = GOLD["perf_model_ab34"]["grids"]
    assert g["fast"][0] * g["fast"][1] == GOLD["perf_model_ab34"]["n_f"]
    assert g["slow"][0] * g["slow"][1] == GOLD["perf_model_ab34"]["n_s"]


@pytest.mark.parametrize("key", ["perf_model_ab34", "perf_model_ab45"])
def test_rhs_counts_and_speedups_match_paper_table(key):
    d = GOLD[key]
    nf, ns = d["n_f"], d["n_s"]
    dt = 0.0217                       # RK4's stable step; only t / dt_RK4 = 1 enters
    rk4 = perfmodel.rhs_evals_rk4(dt, dt, nf, ns)
    assert rk4 == pytest.approx(d["rk4_total"], rel=1e-12)
    for sr, (r, total, red, su) in enumerate(zip(d["r_rk4"], d["total_rhs"], d["pct_reduction"], d["su"]), 1):
        ab = perfmodel.rhs_evals_ab(dt, dt, r, sr, nf, ns)
        # the printed r_RK4 carry three digits, the totals were formed from unrounded ratios
        assert ab == pytest.approx(total, rel=3e-3), (key, sr)
        assert 100.0 * (1.0 - ab / rk4) == pytest.approx(red, abs=0.3), (key, sr)
        assert round(perfmodel.speedup(dt, dt, r, sr, nf, ns), 2) == pytest.approx(su, abs=0.011), (key, sr)


def test_a_wrong_model_fails_the_table():
    """Dropping RK4's four stages, or counting the slow grid SR times, moves
    the totals far outside the tolerance used above."""
    d = GOLD["perf_model_ab34"]
    nf, ns = d["n_f"], d["n_s"]
    sr, r, total = 4, d["r_rk4"][3], d["total_rhs"][3]
    assert abs((sr * nf + sr * ns) / r / total - 1.0) > 0.3
    assert abs(perfmodel.rhs_evals_rk4(1.0, 1.0, nf, ns) / 4.0 / d["rk4_total"] - 1.0) > 0.5


def test_macrostep_count_generalises_the_two_level_count():
    assert perfmodel.rhs_evals_per_macrostep([4, 1], [4840, 3721]) == 4 * 4840 + 3721
    assert perfmodel.rhs_evals_per_macrostep([1, 2, 2, 4], [10, 20, 30, 40]) == 10 + 40 + 60 + 160


def test_cylinder_points_per_macrostep_from_oracle_blanking():
    """Point evaluations per macrostep of the cylinder problem with the
    oracle's own blanking: the quantity the throughput metric counts."""
    import workloads
    from oracle import overset
    wl = workloads.cylinder()
    act = [int(overset.blank(g).sum()) for g in wl.grids]
    n = perfmodel.rhs_evals_per_macrostep([g.rate for g in wl.grids], act)
    assert act[1] == 256 * 128
    assert n == act[0] + 4 * act[1]
    assert 250_000 < act[0] < 262_144

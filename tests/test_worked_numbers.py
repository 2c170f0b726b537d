"""Worked numbers printed in the paper (tests/golden/worked_numbers.json)
against the sizing helpers."""
import json
import math
import os

from paper_2306_01301_amd import sizing

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_numbers.json")))


def test_resolution_rules():
    g = GOLD["resolution"]
    dc = math.hypot(g["box_forward_m"], g["box_side_m"])
    assert round(dc, 1) == g["corner_distance_m"]
    assert round(math.degrees(g["cell_m"] / dc), 1) == g["dtheta_deg_approx"]
    n = sizing.headings_for_turns(g["turn_radius_m"], g["cell_m"])
    assert math.ceil(n) == g["min_headings_turns"]
    assert sizing.headings_for_collision(dc, g["cell_m"]) < n <= g["cube_side"]


def test_sufficient_transition_cost():
    g = GOLD["sufficient_transition_cost"]
    R, dth = g["turn_radius_m"], 2 * math.pi / g["n_theta"]
    total = sizing.sufficient_transition_cost(g["dx_m"], g["dy_m"], dth, R)
    terms = [g["dx_m"], R * dth, total - g["dx_m"] - R * dth]
    for got, want in zip(terms, g["terms_m"]):
        assert abs(got - want) < 0.005
    assert round(total, 1) == g["total_m"] <= g["natural_cost_m"]
    t = GOLD["transition_cost_example"]
    assert abs(t["v_max_mps"] * t["t_w_s"] - t["d_w_m"]) < 1e-9


def test_complexity_tables():
    g = GOLD["complexity"]
    nr = 2.0 ** g["log2_nr"]
    piano = sizing.graph_complexity("piano", nr)
    assert round(piano) == g["piano"]
    assert int(sizing.graph_complexity("compact", nr)) == g["compact"]
    assert int(sizing.graph_complexity("star", nr)) == g["star"]
    assert sizing.kernel_complexity(g["n_cycles"]) == g["kernel"]
    for k, want in g["relative"].items():
        # the table divides its own truncated entries
        val = (sizing.kernel_complexity(g["n_cycles"]) if k == "kernel" else int(sizing.graph_complexity(k, nr)))
        assert round(val / round(piano), 2) == want
    m = GOLD["memory"]
    for k in ("piano", "compact", "star"):
        assert sizing.memory_volumes(k) == m[k]
    assert sizing.memory_volumes("star", kernel_style=True) == m["kernel"]


def test_update_count():
    assert sizing.pose_updates(512, 512, 20) == 6 * 20 * 512 ** 3
    assert sizing.sweep_bytes(512, 512, 20) == 9 * 6 * 20 * 512 ** 3

"""The paper's printed parameter tables (tests/golden/*.json, each with its
citation) against the presets and bounds the workloads use, and the oracle
on those presets."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2607_06499_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_fixtures_carry_citations():
    for name in sorted(os.listdir(GOLDEN)):
        if name.endswith(".json"):
            assert _load(name)["citation"].startswith("Sec. "), name


def test_unicycle_bounds_are_the_papers():
    g = _load("simulation_parameters.json")
    assert W.TABLE1_UMAX[:2] == [g["linear_velocity_bound"], g["angular_velocity_bound"]]
    assert W.TABLE1_UMIN[:2] == [-g["linear_velocity_bound"], -g["angular_velocity_bound"]]


@pytest.mark.parametrize("scenario", [1, 2])
def test_unicycle_preset_matches_simulation_table(scenario):
    g = _load("simulation_parameters.json")
    spec = W.paper_unicycle_preset(scenario).spec
    f32 = lambda x: float(np.float32(x))
    assert spec.num_samples == g["K"] and spec.horizon == g["N"]
    assert spec.dt == f32(g["dt"])
    assert spec.lam == f32(g[f"lambda_scenario_{scenario}"])
    assert spec.Q[:3] == [f32(v) for v in g["Q_diag"]]
    assert spec.Qf[:3] == [f32(v) for v in g["H_diag"]]
    assert spec.R[:2] == [0.0, 0.0]
    assert spec.u_max[:2] == [f32(g["linear_velocity_bound"]), f32(g["angular_velocity_bound"])]
    if scenario == 2:
        s = W.paper_unicycle_preset(2)
        assert abs(float(np.linalg.norm(s.field.v[0])) - g["scenario_2_obstacle_speed"]) < 1e-12


def test_arm_preset_matches_real_world_table():
    g = _load("real_parameters.json")
    spec = W.paper_arm_preset().spec
    f32 = lambda x: float(np.float32(x))
    assert spec.num_samples == g["K"] and spec.horizon == g["N"]
    assert spec.dt == f32(g["dt"]) and spec.lam == f32(g["lambda"])
    assert spec.dbscan_eps == f32(g["dbscan_eps"])
    assert spec.u_max == [f32(g["joint_velocity_bound"])] * 6
    assert spec.u_min == [-f32(g["joint_velocity_bound"])] * 6
    assert spec.q_limit == [f32(g["joint_position_bound"])] * 6
    assert spec.Q[:3] == [f32(g["w_p"]), f32(g["w_R"]), f32(g["w_c"])]
    assert spec.Qf[:3] == spec.Q[:3]
    assert spec.flags == W.FLAG_POSE_COST
    assert abs(g["joint_position_bound"] - 2 * math.pi) < 1e-15


@pytest.mark.parametrize("make", [lambda: W.paper_unicycle_preset(1), lambda: W.paper_unicycle_preset(2),
                                  W.paper_arm_preset])
def test_oracle_on_presets_takes_the_clustering_branch(make):
    s = make()
    o = oracle.replan(s.spec, s.x0, s.U0, s.obstacles)
    assert o["branch"] == 0 and o["n_clusters"] >= 1
    assert np.all(np.abs(o["u_out"]) <= np.array(s.spec.u_max[: s.spec.m]) + 1e-12)
    assert abs(float(np.sum(o["weight"])) - 1.0) < 1e-9

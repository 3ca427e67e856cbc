"""Pins of the oracle's cluster statistics and selection on given labels
(Alg. 1 [Cluster stats] and [Selection]; Eq. (14) static, Eq. (16)-(18)
dynamic): synthetic clusters with known means and directions."""
import math

import numpy as np
import pytest

from paper_2607_06499_amd import workloads as W


def _spec(mode=W.STATIC, H=5):
    return W.PlannerSpec(num_samples=64, scene_mode=mode, history_len=H, dt=0.1).rounded()


def _unit(a):
    return np.array([math.cos(a), math.sin(a)])


def test_static_rule_minimum_mean_cost(orc):
    lab = np.array([0, 0, 1, 1, 1, -1, 2, 2])
    S = np.array([4.0, 6.0, 1.0, 2.0, 3.0, -100.0, 2.5, 2.5])
    g = np.array([_unit(0.1 * i) for i in range(8)])
    r = orc.select_cluster(_spec(), lab, S, g, np.zeros((0, 3)))
    assert r["rule"] == 0 and r["selected"] == 1
    assert np.allclose(r["c_mean_cost"], [5.0, 2.0, 2.5], atol=1e-15)
    assert list(r["c_size"]) == [2, 3, 2] and r["selected_size"] == 3
    assert r["margin"] == pytest.approx(0.5, abs=1e-15)
    # normalised mean directions, Eq. (16): noise excluded
    for c in range(3):
        v = g[lab == c].mean(0)
        assert np.allclose(r["c_dir"][c], v / (np.linalg.norm(v) + 1e-6), atol=1e-12)


def test_static_tie_goes_to_lowest_label(orc):
    lab = np.array([0, 1, 2])
    S = np.array([3.0, 1.0, 1.0])
    g = np.array([_unit(0.0), _unit(1.0), _unit(2.0)])
    r = orc.select_cluster(_spec(), lab, S, g, np.zeros((0, 3)))
    assert r["selected"] == 1 and r["margin"] == 0.0


def test_dynamic_rule_most_opposite_direction(orc):
    # obstacle 1 moves along +x at 0.4 m/s (constant velocity history)
    dt = float(np.float32(0.1))
    o_now = np.array([[5.0, 5.0, 0.3], [2.0, 1.0, 0.4]])
    v = np.array([0.4, 0.0])
    hist = np.stack([o_now[:, :2] - h * dt * np.array([[0.0, 0.0], v]) for h in range(5)])
    lab = np.array([0, 0, 1, 1, 2])
    g = np.array([_unit(0.0), _unit(0.2), _unit(math.pi), _unit(math.pi - 0.1), _unit(math.pi / 2)])
    S = np.array([1.0, 1.0, 9.0, 9.0, 0.0])
    r = orc.select_cluster(_spec(W.DYNAMIC), lab, S, g, o_now, hist=hist, closest=1)
    assert r["rule"] == 1 and r["h_used"] == 5
    assert np.allclose(r["v_obs"], v, atol=1e-12)
    assert np.allclose(r["v_obs_hat"], v / (0.4 + 1e-6), atol=1e-12)
    # cluster 1 points against the motion although its cost is the highest
    assert r["selected"] == 1
    dots = r["c_dir"] @ r["v_obs_hat"]
    assert r["margin"] == pytest.approx(np.sort(dots)[1] - np.sort(dots)[0], abs=1e-12)


def test_dynamic_mirror_tie_and_preconditions(orc):
    dt = float(np.float32(0.1))
    o_now = np.array([[0.0, 0.0, 0.3]])
    v = np.array([0.0, 0.5])
    hist = np.stack([o_now[:, :2] - h * dt * v for h in range(3)])
    # two clusters mirrored about the motion axis: equal dot products
    lab = np.array([0, 1])
    g = np.array([_unit(-0.7), _unit(math.pi + 0.7)])
    g[1] = [-g[0][0], g[0][1]]
    S = np.array([5.0, 1.0])
    r = orc.select_cluster(_spec(W.DYNAMIC, H=3), lab, S, g, o_now, hist=hist, closest=0)
    assert r["rule"] == 1 and r["selected"] == 0 and r["margin"] == 0.0
    # one observation only: static rule, status bit set
    r = orc.select_cluster(_spec(W.DYNAMIC, H=3), lab, S, g, o_now, hist=hist[:1], closest=0)
    assert r["rule"] == 0 and r["status"] & orc.ST_DYN_STATIC and r["selected"] == 1
    # a resting obstacle: static rule
    still = np.stack([o_now[:, :2]] * 3)
    r = orc.select_cluster(_spec(W.DYNAMIC, H=3), lab, S, g, o_now, hist=still, closest=0)
    assert r["rule"] == 0 and r["status"] & orc.ST_DYN_STATIC


def test_select_step_agrees_with_full_replan(orc):
    s = W.unicycle_static_ahead(1)
    r = orc.replan(s.spec, s.x0, s.U0, s.obstacles)
    assert r["branch"] == 0 and r["n_clusters"] >= 2
    q = orc.select_cluster(s.spec, r["label"], r["S"][r["v_idx"]], r["g"], s.obstacles,
                           closest=r["closest"])
    assert q["selected"] == r["selected"] and q["rule"] == r["rule"]
    assert np.array_equal(q["c_mean_cost"], r["c_mean_cost"])
    assert np.array_equal(q["c_dir"], r["c_dir"]) and np.array_equal(q["c_size"], r["c_size"])

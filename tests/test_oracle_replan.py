"""Pins of the oracle's full replan (Alg. 1): branches, reference point,
features, selection rules, obstacle-motion estimate, update and shift."""
import math

import numpy as np
import pytest

from paper_2607_06499_amd import workloads as W


def _replan(orc, scene, hist=None, step=0, U=None):
    return orc.replan(scene.spec, scene.x0, scene.U0 if U is None else U, scene.obstacles,
                      hist=hist, step=step)


def test_no_obstacles_is_plain_mppi(orc):
    s = W.random_scene(3, n_obs=0, clamp=False)
    r = _replan(orc, s)
    assert r["branch"] == 1 and r["status"] & orc.ST_FALLBACK
    # applied perturbations are the drawn noise; every rollout is weighted
    for k in (0, 17, s.spec.num_samples - 1):
        _, eps = orc.rollout_noise(s.spec, 0, k)
        assert np.allclose(r["eps_eff"][k], eps, atol=1e-12)
        sim = orc.simulate(s.spec, s.x0, s.U0 + eps, np.zeros((0, 3)))
        assert r["S"][k] == pytest.approx(sim["S"], rel=1e-12)
    assert r["weight"].sum() == pytest.approx(1.0, abs=1e-12)
    assert np.all(r["weight"] > 0)
    Un, _, _ = orc.weighted_update(np.arange(s.spec.num_samples), r["S"], r["eps_eff"],
                                   s.spec.lam, s.U0)
    assert np.allclose(r["U_new"], Un, atol=1e-12)


def test_zero_noise_reproduces_nominal(orc):
    s = W.random_scene(4, n_obs=0, clamp=False)
    spec = s.spec.replace(noise_chol=[0.0] * 36)
    r = orc.replan(spec, s.x0, s.U0, s.obstacles)
    sim = orc.simulate(spec, s.x0, s.U0, np.zeros((0, 3)))
    assert np.allclose(r["p_term"], sim["p_term"][None, :], atol=0)
    assert np.allclose(r["S"], sim["S"], atol=0)
    assert np.allclose(r["U_new"], s.U0, atol=0)


def test_clamp_and_applied_perturbation(orc):
    s = W.random_scene(5, n_obs=2, clamp=True)
    r = _replan(orc, s)
    lo, hi = np.array(s.spec.u_min[:2]), np.array(s.spec.u_max[:2])
    ut = s.U0[None] + r["eps_eff"]
    assert np.all(ut >= lo - 1e-12) and np.all(ut <= hi + 1e-12)
    for k in range(0, s.spec.num_samples, 37):
        _, eps = orc.rollout_noise(s.spec, 0, k)
        raw = s.U0 + eps
        inside = (raw > lo) & (raw < hi)
        assert np.allclose(r["eps_eff"][k][inside], eps[inside], atol=1e-12)
        assert np.allclose(ut[k][~inside], np.clip(raw, lo, hi)[~inside], atol=1e-12)


def _ahead_scene(seed=1, D=1.5, rad=0.3, v=0.7):
    """unicycle_static robot with a single obstacle D m straight ahead and a constant
    nominal speed: the feasible rollouts split into a left and a right group."""
    s = W.unicycle_static_ahead(seed)
    h = math.pi / 4
    s.field.c = (s.x0[:2] + D * np.array([math.cos(h), math.sin(h)]))[None]
    s.field.r = np.array([rad])
    s.field.v = np.zeros((1, 2))
    s.U0 = np.zeros_like(s.U0)
    s.U0[:, 0] = v
    return s


def _cluster_scene(orc, seed=1):
    s = _ahead_scene(seed)
    r = _replan(orc, s)
    assert r["branch"] == 0 and r["n_clusters"] >= 2
    return s, r


def test_reference_point_and_features(orc):
    for mode in (W.REF_TERMINAL, W.REF_FIRST_CONTACT):
        s = W.unicycle_static_ahead(1)
        s.spec = s.spec.replace(ref_mode=mode)
        r = _replan(orc, s)
        assert r["branch"] == 0
        col = r["col"].astype(bool)
        A = col & (r["first_obs"] == r["closest"])
        assert A.any() and r["n_ref"] == A.sum()
        src = r["p_term"] if mode == W.REF_TERMINAL else r["p_first"]
        assert np.allclose(r["ref_point"], src[A].mean(0), atol=1e-12)
        V = r["v_idx"]
        assert np.array_equal(V, np.nonzero(~col)[0])
        d = r["p_term"][V] - r["ref_point"]
        nz = np.linalg.norm(r["z"], axis=1)
        assert np.all(nz < 1.0)
        # z is d scaled by 1/(|d| + eps): parallel to d with |z| = |d|/(|d|+eps)
        cross = d[:, 0] * r["z"][:, 1] - d[:, 1] * r["z"][:, 0]
        assert np.max(np.abs(cross)) < 1e-12
        assert np.all(np.sum(d * r["z"], axis=1) > 0)  # same direction, not opposite
        nd = np.linalg.norm(d, axis=1)
        assert np.allclose(nz, nd / (nd + s.spec.norm_eps), atol=1e-14)
        e = r["p_term"][V] - s.x0[:2]
        ng = np.linalg.norm(r["g"], axis=1)
        assert np.allclose(ng, np.linalg.norm(e, axis=1) / (np.linalg.norm(e, axis=1) + 1e-6), rtol=1e-6)


def test_reference_point_uses_closest_obstacle_hits(orc):
    # a second obstacle beside the path catches some rollouts first: only the
    # rollouts whose first contact is the closest obstacle enter the mean
    s = _ahead_scene(D=1.2, rad=0.25)
    h = math.pi / 4
    left = np.array([-math.sin(h), math.cos(h)])
    fwd = np.array([math.cos(h), math.sin(h)])
    side = s.x0[:2] + 1.3 * fwd + 0.55 * left
    s.field.c = np.concatenate([s.field.c, side[None]])
    s.field.r = np.array([0.25, 0.25])
    s.field.v = np.zeros((2, 2))
    r = _replan(orc, s)
    col = r["col"].astype(bool)
    assert r["closest"] == 0
    A = col & (r["first_obs"] == 0)
    other = col & (r["first_obs"] == 1)
    assert A.sum() > 10 and other.sum() > 10
    assert r["n_ref"] == A.sum()
    assert np.allclose(r["ref_point"], r["p_term"][A].mean(0), atol=1e-12)
    assert not np.allclose(r["ref_point"], r["p_term"][col].mean(0), atol=1e-3)


def test_reference_point_falls_back_to_all_colliding(orc):
    # the closest obstacle is off to the side and never hit: A is empty and the
    # reference point is the mean over every colliding rollout (Eq. (11))
    s = W.unicycle_static_ahead(1)
    fld = s.field
    fld.c = np.concatenate([[s.x0[:2] + np.array([0.45, -0.45])], fld.c])
    fld.r = np.concatenate([[0.05], fld.r])
    fld.v = np.concatenate([[np.zeros(2)], fld.v])
    r = _replan(orc, s)
    assert r["closest"] == 0
    col = r["col"].astype(bool)
    assert not np.any(col & (r["first_obs"] == 0))
    assert r["n_ref"] == col.sum()
    assert np.allclose(r["ref_point"], r["p_term"][col].mean(0), atol=1e-12)


def test_static_selection_minimum_mean_cost(orc):
    s, r = _cluster_scene(orc)
    M = r["n_clusters"]
    assert r["selected"] == int(np.argmin(r["c_mean_cost"][:M].astype(np.float32)))
    labs = r["label"]
    S = r["S"][r["v_idx"]]
    for c in range(M):
        assert r["c_mean_cost"][c] == pytest.approx(S[labs == c].mean(), rel=1e-12)
        assert r["c_size"][c] == np.sum(labs == c)
    # the update uses only the selected cluster
    sel = r["v_idx"][labs == r["selected"]]
    assert np.all(r["weight"][sel] > 0)
    assert r["weight"].sum() == pytest.approx(1.0, abs=1e-12)
    assert np.count_nonzero(r["weight"]) == len(sel)
    assert np.allclose(r["U_new"], s.U0 + np.tensordot(r["weight"], r["eps_eff"], axes=(0, 0)),
                       atol=1e-12)


def test_static_selection_prefers_goal_side(orc):
    # obstacle straight ahead, goal off to the left of the heading: the chosen
    # cluster passes the obstacle on the goal's side
    for side in (+1, -1):
        s = _ahead_scene()
        h = math.pi / 4
        left = np.array([-math.sin(h), math.cos(h)])
        goal = s.x0[:2] + 4.0 * np.array([math.cos(h), math.sin(h)]) + side * 3.0 * left
        s.spec = s.spec.replace(goal=[goal[0], goal[1], 0, 0, 0, 0])
        r = _replan(orc, s)
        assert r["branch"] == 0 and r["n_clusters"] >= 2
        sel = r["v_idx"][r["label"] == r["selected"]]
        lateral = (r["p_term"][sel] - s.x0[:2]) @ left
        assert np.sign(np.mean(lateral)) == side


def test_dynamic_selection_opposes_obstacle_motion(orc):
    # the obstacle ahead moves across the path; the chosen cluster is the one
    # whose mean direction has the smallest dot product with its motion
    for side in (+1, -1):
        s = _ahead_scene()
        s.spec = s.spec.replace(scene_mode=W.DYNAMIC, history_len=3)
        h = math.pi / 4
        left = np.array([-math.sin(h), math.cos(h)])
        s.field.v = (side * 0.5 * left)[None]
        dt = s.spec.dt
        cur = s.field.positions()
        hist = np.stack([cur - i * dt * s.field.v.astype(np.float32) for i in range(3)])
        r = _replan(orc, s, hist=hist)
        assert r["branch"] == 0 and r["rule"] == 1 and r["n_clusters"] >= 2
        vh = r["v_obs_hat"]
        dots = r["c_dir"][: r["n_clusters"]] @ vh
        assert r["selected"] == int(np.argmin(dots.astype(np.float32)))
        sel = r["v_idx"][r["label"] == r["selected"]]
        lateral = (r["p_term"][sel] - s.x0[:2]) @ left
        assert np.sign(np.mean(lateral)) == -side


def test_obstacle_velocity_estimate(orc):
    rng = np.random.default_rng(0)
    dt = 0.05
    v = np.array([0.3, -0.8])
    o0 = rng.normal(size=(4, 2))
    hist = np.stack([o0 - h * dt * v for h in range(6)])   # constant velocity, newest first
    for H in (2, 3, 5, 6):
        assert np.allclose(orc.obstacle_velocity(hist, 2, H, dt), v, atol=1e-12)
    # telescoping: the mean of H'-1 differences is (o_t - o_{t-H'+1}) / ((H'-1) dt)
    hist = rng.normal(size=(7, 4, 3))
    for H in (2, 4, 7, 9):
        Hp = min(H, 7)
        exp = (hist[0, 1] - hist[Hp - 1, 1]) / ((Hp - 1) * dt)
        assert np.allclose(orc.obstacle_velocity(hist, 1, H, dt), exp, atol=1e-12)
    assert np.all(orc.obstacle_velocity(hist[:1], 1, 5, dt) == 0)


def test_dynamic_rule_needs_history_and_motion(orc):
    s = W.unicycle_static_ahead(1)
    s.spec = s.spec.replace(scene_mode=W.DYNAMIC)
    r = _replan(orc, s)  # one observation only
    assert r["rule"] == 0 and r["status"] & orc.ST_DYN_STATIC
    cur = s.field.positions()
    r = _replan(orc, s, hist=np.stack([cur, cur]))  # obstacle not moving
    assert r["rule"] == 0 and r["status"] & orc.ST_DYN_STATIC


def test_all_collide_and_no_cluster(orc):
    s = W.unicycle_static_ahead(1)
    s.field.c[0] = s.x0[:2]
    s.field.r[0] = 5.0
    r = _replan(orc, s)
    assert r["branch"] == 2 and r["status"] & orc.ST_ALL_COLLIDE and r["n_feas"] == 0
    assert np.count_nonzero(r["weight"]) == s.spec.num_samples
    s = W.unicycle_static_ahead(1)
    s.spec = s.spec.replace(dbscan_min_pts=100000)
    r = _replan(orc, s)
    assert r["branch"] == 0 and r["n_clusters"] == 0 and r["status"] & orc.ST_NO_CLUSTER
    assert np.count_nonzero(r["weight"]) == r["n_feas"]
    assert np.all(r["weight"][r["v_idx"]] > 0)


def test_shift_and_output(orc):
    s, r = _cluster_scene(orc, 2)
    assert np.array_equal(r["u_out"], r["U_new"][0])
    assert np.array_equal(r["U_next"][:-1], r["U_new"][1:])
    assert np.array_equal(r["U_next"][-1], r["U_new"][-1])


def test_nonfinite_input_is_a_noop(orc):
    s = W.unicycle_static_ahead(1)
    x = s.x0.copy()
    x[1] = np.nan
    r = orc.replan(s.spec, x, s.U0, s.obstacles)
    assert r["status"] & orc.ST_NONFINITE
    assert np.array_equal(r["U_new"], s.U0) and np.array_equal(r["U_next"], s.U0)


def test_arm_replan_structure(orc):
    s = W.random_scene(2, dynamics=W.ARM6, num_samples=256, horizon=16, n_obs=10)
    r = _replan(orc, s)
    assert r["p_term"].shape == (256, 3)
    # terminal point is the forward kinematics of the integrated joints
    dh = np.asarray(s.spec.dh).reshape(6, 4)
    for k in (0, 100, 255):
        q = s.x0[:6] + s.spec.dt * (s.U0 + r["eps_eff"][k]).sum(0)
        org, _ = orc.arm_frames(q, dh)
        assert np.allclose(r["p_term"][k], org[6], atol=1e-12)
    assert r["weight"].sum() == pytest.approx(1.0, abs=1e-12)

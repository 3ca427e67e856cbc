"""GPU parity: the HIP replan path (through the C-ABI) against the FP64
oracle on the same seeded inputs."""
import math

import numpy as np
import pytest

import oracle
from paper_2607_06499_amd import workloads as W
from tests import harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not H.gpu_ok():
        pytest.skip("no GPU")
    from paper_2607_06499_amd import binding

    binding.load()


def _planner(spec):
    from paper_2607_06499_amd import binding as B

    return B.Planner(spec)


def _set_U(pl, U):
    pl.set_nominal(H.to_dev(np.asarray(U, np.float32)))


# ------------------------------------------------------------------ noise
@pytest.mark.parametrize("dyn,N,K,step,seed", [(W.UNICYCLE, 23, 301, 7, 5), (W.ARM6, 13, 97, 123456, 2**40 + 3),
                                               (W.UNICYCLE, 1, 5, 0, 0)])
def test_noise_words_bit_exact(dyn, N, K, step, seed):
    spec = W.PlannerSpec(dynamics=dyn, horizon=N, num_samples=K, seed=seed, stream_id=11,
                         noise_chol=W.diag_chol([1.0] * 6, 2 if dyn == 0 else 6),
                         dh=W.arm_dh([0.2] * 6)).rounded()
    pl = _planner(spec)
    words, gauss = pl.stage_noise(step)
    words = words.cpu().numpy().view(np.uint32)
    gauss = gauss.cpu().numpy()
    m = spec.m
    for k in range(K):
        ref = oracle.noise_words(spec, step, k).reshape(-1, 4)
        assert np.array_equal(words[k], ref), k
        g, _ = oracle.rollout_noise(spec, step, k)
        err = np.abs(gauss[k] - g) / np.maximum(np.abs(g), 1.0)
        assert err.max() <= H.GAUSS_TOL, (k, err.max())
    assert gauss.shape == (K, N, m)


# ------------------------------------------------------------------ rollouts
def _compare_rollouts(r, o, spec, check_eps=True):
    """Rollout records: costs, trajectories end points, collision flags."""
    bnd = o["clearance"] <= H.BOUNDARY
    ok = ~bnd
    perr = H.rel_err(r["p_term"], o["p_term"]).max()
    serr = H.rel_err(r["S"], o["S"]).max()
    flips = int(np.sum(r["col"][bnd] != o["col"][bnd]))
    print(f"rollouts: K={spec.num_samples} max p_term err {perr:.2e} max S err {serr:.2e} "
          f"boundary {int(bnd.sum())} flipped {flips}")
    assert np.array_equal(r["col"][ok], o["col"][ok])
    both = ok & (o["col"] == 1)
    assert np.array_equal(r["first_obs"][both], o["first_obs"][both])
    # the pose cost counts contact states, so a boundary flip moves S by w_c
    srows = ok if spec.flags & W.FLAG_POSE_COST else np.ones_like(ok)
    assert H.rel_err(r["S"][srows], o["S"][srows]).max() <= H.TRAJ_RTOL
    assert H.rel_err(r["p_term"], o["p_term"]).max() <= H.TRAJ_RTOL
    if both.any():
        assert H.rel_err(r["p_first"][both], o["p_first"][both]).max() <= H.TRAJ_RTOL
    if check_eps:
        e = np.abs(r["eps_eff"] - o["eps_eff"]) / np.maximum(np.abs(o["eps_eff"]), 1.0)
        assert e.max() <= 1e-5
    return bnd


SCENES = [
    ("random_uni", lambda: W.random_scene(1, num_samples=1000, horizon=30, n_obs=7)),
    ("random_uni_noclamp", lambda: W.random_scene(2, num_samples=777, horizon=50, n_obs=12, clamp=False)),
    ("random_uni_short", lambda: W.random_scene(3, num_samples=513, horizon=9, n_obs=3)),
    ("unicycle_static_ahead", lambda: W.unicycle_static_ahead(1)),
    ("unicycle_dynamic_ahead", lambda: W.unicycle_dynamic_ahead(2, num_samples=2048)),
    ("random_arm", lambda: W.random_scene(4, dynamics=W.ARM6, num_samples=600, horizon=20, n_obs=10)),
    ("random_arm_noclamp", lambda: W.random_scene(5, dynamics=W.ARM6, num_samples=301, horizon=32,
                                                  n_obs=16, clamp=False)),
]


@pytest.mark.parametrize("name,make", SCENES, ids=[s[0] for s in SCENES])
def test_rollouts_match_oracle(name, make):
    s = make()
    pl = _planner(s.spec)
    _set_U(pl, s.U0)
    r = H.gpu_replan(pl, s.x0, s.obstacles)
    o = oracle.replan(s.spec, s.x0, s.U0, s.obstacles)
    _compare_rollouts(r, o, s.spec)


# ------------------------------------------------------------------ stages after the rollouts
def _fp32_records(o):
    return {k: np.asarray(o[k], np.float32 if o[k].dtype == np.float64 else np.int32)
            for k in ("S", "col", "first_obs", "p_term", "p_first", "eps_eff")}


def _resolve(spec, x, U, obs, hist, step, o, r, bnd):
    """The oracle's replan with the decisions that lie inside their flagged
    bands taken the way the GPU took them: collision flags (and first contacts)
    of rollouts at a contact boundary, and o* when the two smallest surface
    clearances are within FP32 rounding of each other.  Everything else stays
    the oracle's own FP64 result."""
    inf = r["info"]
    flips = bnd & ((r["col"] != o["col"]) | ((r["col"] == 1) & (r["first_obs"] != o["first_obs"])))
    pose = bool(spec.flags & W.FLAG_POSE_COST)
    closest = None
    if inf["closest"] != o["closest"]:
        assert o["closest_margin"] <= 1e-5 * (1.0 + abs(o["closest_margin"])), (
            inf["closest"], o["closest"], o["closest_margin"])
        closest = inf["closest"]
    if not flips.any() and closest is None:
        return o, 0
    rec = {k: np.array(o[k], copy=True) for k in ("S", "col", "first_obs", "p_term", "p_first", "eps_eff")}
    rec["col"][flips] = r["col"][flips]
    rec["first_obs"][flips] = r["first_obs"][flips]
    rec["p_first"][flips] = r["p_first"][flips]
    if pose:  # a contact state moves the pose cost by w_c
        rec["S"][bnd] = r["S"][bnd]
    o2 = oracle.replan(spec, x, U, obs, hist, step=step, rollouts=rec, closest=closest)
    o2["clearance"] = o["clearance"]
    return o2, int(flips.sum())


def _check_post(r, o, spec, U, obs, hist=None, tag=""):
    """Every stage after the rollouts of one GPU replan against the oracle
    (o: the oracle's replan on the same inputs, flagged decisions resolved by
    _resolve).  Stage by stage on the GPU's own inputs to the stage, and end
    to end against the oracle's values.  Returns the counts it found."""
    inf = r["info"]
    st = dict(branch=inf["branch"])
    assert inf["branch"] == o["branch"], tag
    assert inf["n_collide"] == o["n_col"] and inf["n_feasible"] == o["n_feas"], tag
    U = np.asarray(U, np.float64)
    emax = max(1.0, float(np.abs(r["eps_eff"]).max()))
    if o["branch"] != 0:
        assert inf["status"] == o["status"], (tag, inf["status"], o["status"])
        # Eq. (6)-(7) over every rollout, on the GPU's costs and perturbations
        Un, _, _ = oracle.weighted_update(np.arange(spec.num_samples), r["S"], r["eps_eff"], spec.lam, U)
        assert np.abs(r["U_new"] - Un).max() <= 1e-4 * emax, tag
        dS = np.abs(r["S"].astype(np.float64) - o["S"]).max()
        eo = np.abs(o["eps_eff"]).max()
        assert np.all(np.abs(r["U_new"] - o["U_new"]) <= 2.0 * (dS / spec.lam) * eo + 1e-4 * emax), tag
        return st
    assert inf["n_ref"] == o["n_ref"], tag
    assert inf["closest"] == o["closest"], tag
    assert np.array_equal(r["v_idx"], o["v_idx"]), tag
    assert H.rel_err(inf["ref_point"][: spec.p], o["ref_point"]).max() <= 1e-5, tag
    # z = d / |d| amplifies the FP32 error of d = p_term - ref by 2 / |d|
    slack = H.feature_slack(o["p_term"][o["v_idx"]], o["ref_point"])
    assert np.all(np.abs(r["z"] - o["z"]).max(axis=1) <= slack), tag
    assert np.abs(r["g"] - o["g"]).max() <= 2e-5, tag
    eps = float(np.float32(spec.dbscan_eps))
    mp = spec.dbscan_min_pts
    # DBSCAN stage: the definition on the GPU's own features
    zg = np.asarray(r["z"], np.float64)
    olab, _, _, oM = oracle.dbscan(zg, eps, mp)
    ds = H.dbscan_check(zg, eps, mp, r["ncount"], r["label"], 0.5 * H.STAGE_BAND * eps, exact_ref=olab,
                        tag=tag + " dbscan stage")
    M = inf["n_clusters"]
    assert M == (int(r["label"].max()) + 1 if len(r["label"]) and r["label"].max() >= 0 else 0), tag
    # end to end: against the oracle's features, pairs within the FP32 error
    # of the features (and the 1e-4 eps band) left free
    ms = H.feature_slack_measured(r["p_term"][r["v_idx"]], o["p_term"][o["v_idx"]],
                                  inf["ref_point"][: spec.p], o["ref_point"])
    assert np.all(np.abs(r["z"] - o["z"]).max(axis=1) <= ms), tag
    de = H.dbscan_check(o["z"], eps, mp, r["ncount"], r["label"], 0.5 * H.PAIR_BAND * eps + ms,
                        exact_ref=o["label"], tag=tag + " dbscan end to end")
    st.update(V=len(r["label"]), M=M, stage_flagged_pairs=ds["flagged_pairs"],
              stage_differing=ds["differing"], e2e_flagged_pairs=de["flagged_pairs"],
              e2e_flagged_points=de["flagged_points"], e2e_differing=de["differing"])
    print(f"{tag}: V={st['V']} M={M} stage: {ds['flagged_pairs']} flagged pairs, "
          f"{ds['differing']} labels differ; end to end: {de['flagged_pairs']} flagged pairs on "
          f"{de['flagged_points']} points, {de['differing']} labels differ")
    Sg = np.asarray(r["S"], np.float64)
    if M == 0:
        assert inf["status"] == 4, (tag, inf["status"])
        upd_set = r["v_idx"]
    else:
        # statistics and selection on the GPU's labels, costs and directions
        q = oracle.select_cluster(spec, r["label"], Sg[r["v_idx"]], r["g"], obs, hist=hist,
                                  closest=inf["closest"])
        assert np.array_equal(r["c_size"], q["c_size"]), tag
        assert H.rel_err(r["c_mean_cost"], q["c_mean_cost"]).max() <= 1e-5, tag
        assert np.abs(r["c_dir"] - q["c_dir"]).max() <= 2e-5, tag
        assert inf["rule"] == q["rule"], tag
        assert inf["status"] == q["status"], (tag, inf["status"], q["status"])
        assert np.abs(inf["v_obs"][: spec.p] - q["v_obs"]).max() <= 1e-5 * max(1.0, np.abs(q["v_obs"]).max()), tag
        assert np.abs(inf["v_obs_hat"][: spec.p] - q["v_obs_hat"]).max() <= 1e-5, tag
        key = q["c_mean_cost"][q["selected"]] if q["rule"] == 0 else 1.0
        near_tie = np.isfinite(q["margin"]) and abs(q["margin"]) <= 1e-4 * max(1.0, abs(key))
        if not near_tie:
            assert inf["selected"] == q["selected"], (tag, inf["selected"], q["selected"])
        st.update(rule=q["rule"], selected=inf["selected"], near_tie=bool(near_tie))
        upd_set = r["v_idx"][r["label"] == inf["selected"]]
        assert inf["selected_size"] == len(upd_set), tag
        # end to end against the oracle's own clusters when the labels agree
        if np.array_equal(r["label"], o["label"]):
            assert np.array_equal(r["c_size"], o["c_size"]), tag
            assert H.rel_err(r["c_mean_cost"], o["c_mean_cost"]).max() <= 1e-4, tag
            assert np.abs(r["c_dir"] - o["c_dir"]).max() <= 1e-4, tag
            if not near_tie and not (np.isfinite(o["margin"]) and abs(o["margin"]) <= 1e-4 * max(1.0, abs(key))):
                assert inf["selected"] == o["selected"] and inf["rule"] == o["rule"], tag
    # the update of Eq. (19)-(20) on the GPU's set, costs and perturbations
    Un, _, _ = oracle.weighted_update(upd_set, Sg, r["eps_eff"], spec.lam, U)
    assert np.abs(r["U_new"] - Un).max() <= 1e-4 * emax, tag
    # end to end: the weights move by about dS / lambda
    if M == o["n_clusters"] and np.array_equal(r["label"], o["label"]) and inf["selected"] == o["selected"]:
        dS = np.abs(Sg - o["S"]).max()
        eo = np.abs(o["eps_eff"]).max()
        bound = 2.0 * (dS / spec.lam) * eo + 1e-4 * np.maximum(np.abs(o["U_new"]), 1.0)
        assert np.all(np.abs(r["U_new"] - o["U_new"]) <= bound + 1e-4 * eo), tag
        st["e2e_update"] = True
    return st


POST = [
    ("unicycle_static_ahead", lambda: W.unicycle_static_ahead(1)),
    ("unicycle_static_ahead_s3", lambda: W.unicycle_static_ahead(3)),
    ("unicycle_dynamic_ahead", lambda: W.unicycle_dynamic_ahead(2, num_samples=3000)),
    ("random_uni", lambda: W.random_scene(7, num_samples=1500, horizon=40, n_obs=8)),
    ("random_uni_first_contact", lambda: W.random_scene(8, num_samples=900, horizon=30, n_obs=8,
                                                        ref_mode=W.REF_FIRST_CONTACT)),
    ("random_arm", lambda: W.random_scene(26, dynamics=W.ARM6, num_samples=800, horizon=16, n_obs=12)),
    ("arm_ahead", lambda: _arm_ahead(2, num_samples=1024)),
]


@pytest.mark.parametrize("name,make", POST, ids=[s[0] for s in POST])
def test_post_rollout_stages_on_oracle_records(name, make):
    s = make()
    o_full = oracle.replan(s.spec, s.x0, s.U0, s.obstacles)
    rec = _fp32_records(o_full)
    o = oracle.replan(s.spec, s.x0, s.U0, s.obstacles, rollouts=rec)
    pl = _planner(s.spec)
    _set_U(pl, s.U0)
    x = H.to_dev(s.x0)
    obs = H.to_dev(s.obstacles)
    t = {k: H.to_dev(v) for k, v in rec.items()}
    u, U, _ = pl.replan_from_rollouts(x, obs, t["S"], t["col"], t["first_obs"], t["p_term"],
                                      t["p_first"], t["eps_eff"])
    H.torch_mod().cuda.synchronize()
    info = pl.info()
    r = H.collect(pl, info)
    r["U_new"] = U.cpu().numpy()
    st = _check_post(r, o, s.spec, s.U0, s.obstacles, tag=name)
    assert st["branch"] == 0 and st.get("e2e_update"), st
    _check_output_shift(r["U_new"], u.cpu().numpy(), pl.get_nominal().cpu().numpy())


def _check_output_shift(U_new, u_out, U_next):
    """u_out is the first control of the update; the kept sequence is the
    update shifted by one step with the last control repeated."""
    assert np.array_equal(u_out, U_new[0])
    assert np.array_equal(U_next[:-1], U_new[1:])
    assert np.array_equal(U_next[-1], U_new[-1])


# ------------------------------------------------------------------ DBSCAN alone, bit-exact
def _dbscan_cases():
    cases = []
    for name, make in POST:
        s = make()
        o = oracle.replan(s.spec, s.x0, s.U0, s.obstacles)
        if o["branch"] == 0 and o["n_feas"] > 0:
            cases.append((name, np.asarray(o["z"], np.float32), s.spec))
    rng = np.random.default_rng(0)
    # many small separated groups: more than 64 trees (exercises the fallback)
    ang = np.repeat(np.arange(90) * 2 * math.pi / 90, 12) + rng.normal(0, 0.004, 90 * 12)
    z = np.stack([np.cos(ang), np.sin(ang)], 1).astype(np.float32)
    cases.append(("90_groups", z, W.PlannerSpec(num_samples=2000, dbscan_eps=0.03, dbscan_min_pts=5)))
    # duplicates and exact-radius pairs
    z = np.zeros((300, 2), np.float32)
    z[100:200, 0] = np.float32(0.3)
    z[200:] = rng.normal(size=(100, 2)).astype(np.float32)
    cases.append(("dups", z, W.PlannerSpec(num_samples=512, dbscan_eps=0.3, dbscan_min_pts=50)))
    # 3-D features, ragged size
    v = rng.normal(size=(1111, 3))
    v[:500] += 3 * np.array([1, 0, 0])
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    cases.append(("sphere3d", v.astype(np.float32),
                  W.PlannerSpec(dynamics=W.ARM6, num_samples=1200, dbscan_eps=0.35, dbscan_min_pts=16,
                                dh=W.arm_dh([0.2] * 6))))
    # full-size feature sets (64 and 40 tiles): one dense arc of unit
    # features, as the rollouts give, and seven blobs of unequal spread in
    # uniform noise (several hook trees per cluster, long hook chains)
    th = rng.normal(0.7, 0.35, 8184)
    z = np.stack([np.cos(th), np.sin(th)], 1).astype(np.float32)
    cases.append(("arc_8184", z, W.PlannerSpec(num_samples=8192, dbscan_eps=0.25, dbscan_min_pts=20)))
    cen = rng.uniform(-1, 1, (7, 2))
    pts = [cc + rng.normal(0, 0.02 + 0.01 * i, (450 + 40 * i, 2)) for i, cc in enumerate(cen)]
    pts.append(rng.uniform(-1, 1, (5000 - sum(len(q) for q in pts), 2)))
    z = np.concatenate(pts)
    rng.shuffle(z)
    cases.append(("blobs_5000", z.astype(np.float32),
                  W.PlannerSpec(num_samples=5000, dbscan_eps=0.05, dbscan_min_pts=12)))
    return cases


@pytest.mark.parametrize("case", range(12))
def test_stage_dbscan_matches_definition(case):
    """DBSCAN alone on given FP32 features: counts, core flags and labels
    equal the oracle's FP64 definition except on pairs within the FP32
    rounding band of eps, where the result must still be an admissible
    DBSCAN (checked point by point)."""
    cases = _dbscan_cases()
    if case >= len(cases):
        pytest.skip("no such case")
    name, z, spec = cases[case]
    spec = spec.rounded()
    pl = _planner(spec)
    from paper_2607_06499_amd import binding as B

    eps = float(np.float32(spec.dbscan_eps))
    z64 = z.astype(np.float64)
    olab, ocore, ocnt, oM = oracle.dbscan(z64, eps, spec.dbscan_min_pts)
    # the planner's default path, and the bitmap too where the default is
    # the angular windows
    paths = [pl.dbscan_path()] + ([B.DBSCAN_BITMAP] if pl.dbscan_path() == B.DBSCAN_WINDOW else [])
    for path in paths:
        pl.set_dbscan_mode(path)
        lab, cnt, M = pl.stage_dbscan(H.to_dev(z))
        lab = lab.cpu().numpy()
        cnt = cnt.cpu().numpy()
        n_trees, overflow = pl.debug(B.DBG_TREES, 2).cpu().tolist()
        print(f"{name} path {path}: V={len(z)} trees={n_trees} overflow={overflow}")
        st = H.dbscan_check(z64, eps, spec.dbscan_min_pts, cnt, lab, 0.5 * H.STAGE_BAND * eps,
                            exact_ref=olab, tag=name)
        print(f"{name}: {st}")
        if st["flagged_pairs"] == 0:
            assert H.counts_agree(cnt, ocnt, spec.dbscan_min_pts), name
            assert int(M.cpu().item()) == oM, name
        assert int(M.cpu().item()) == (int(lab.max()) + 1 if len(lab) and lab.max() >= 0 else 0)
        if path == B.DBSCAN_WINDOW:
            assert overflow == 0
        else:
            assert overflow == (1 if n_trees > 64 else 0)
            if name == "90_groups":
                assert overflow == 1


def test_stage_dbscan_empty_and_single():
    spec = W.PlannerSpec(num_samples=64, dbscan_eps=0.3, dbscan_min_pts=1).rounded()
    pl = _planner(spec)
    lab, cnt, M = pl.stage_dbscan(H.to_dev(np.zeros((0, 2), np.float32)))
    assert int(M.cpu().item()) == 0 and lab.numel() == 0
    lab, cnt, M = pl.stage_dbscan(H.to_dev(np.ones((1, 2), np.float32)))
    assert int(M.cpu().item()) == 1 and lab.cpu().tolist() == [0]


# ------------------------------------------------------------------ end to end
E2E = [
    ("unicycle_static_ahead", lambda: W.unicycle_static_ahead(1)),
    ("unicycle_static_ahead_s5", lambda: W.unicycle_static_ahead(5)),
    ("unicycle_dynamic_ahead", lambda: W.unicycle_dynamic_ahead(1, num_samples=4096)),
    ("random_uni", lambda: W.random_scene(11, num_samples=2000, horizon=40, n_obs=10)),
    ("random_arm", lambda: W.random_scene(12, dynamics=W.ARM6, num_samples=1000, horizon=24, n_obs=12)),
    ("arm_ahead", lambda: _arm_ahead(3, num_samples=2000)),
    ("no_obstacles", lambda: W.random_scene(13, num_samples=700, horizon=20, n_obs=0)),
    ("paper_unicycle_1", lambda: W.paper_unicycle_preset(1)),
    ("paper_unicycle_2", lambda: W.paper_unicycle_preset(2)),
    ("paper_arm", lambda: W.paper_arm_preset(1)),
    ("paper_arm_s2", lambda: W.paper_arm_preset(2)),
]


@pytest.mark.parametrize("name,make", E2E, ids=[s[0] for s in E2E])
def test_end_to_end_replan(name, make):
    s = make()
    pl = _planner(s.spec)
    _set_U(pl, s.U0)
    r = H.gpu_replan(pl, s.x0, s.obstacles)
    o = oracle.replan(s.spec, s.x0, s.U0, s.obstacles)
    bnd = _compare_rollouts(r, o, s.spec)
    o, nflip = _resolve(s.spec, s.x0, s.U0, s.obstacles, None, 0, o, r, bnd)
    st = _check_post(r, o, s.spec, s.U0, s.obstacles, tag=name)
    print(f"{name}: {nflip} boundary rollouts resolved as the GPU took them; {st}")
    _check_output_shift(r["U_new"], r["u_out"], r["U_next"])


def test_determinism_and_checkpoint():
    s = W.unicycle_static_ahead(2)
    pl = _planner(s.spec)
    _set_U(pl, s.U0)
    state = pl.get_state()
    a = H.gpu_replan(pl, s.x0, s.obstacles)
    b2 = H.gpu_replan(pl, s.x0, s.obstacles)  # next step: different noise
    pl.set_state(state)
    c = H.gpu_replan(pl, s.x0, s.obstacles)
    for k in ("S", "col", "label", "u_out", "U_new", "U_next", "z"):
        assert np.array_equal(a[k], c[k]), k
    assert a["info"]["step"] == 0 and b2["info"]["step"] == 1 and c["info"]["step"] == 0
    assert not np.array_equal(a["S"], b2["S"])


def test_graph_and_direct_launch_agree():
    """The graph replay and direct launches run the same kernels: bitwise
    equal results over a few consecutive replans."""
    from paper_2607_06499_amd import binding as B

    s = W.unicycle_dynamic_ahead(5, num_samples=1500)
    a, b = _planner(s.spec), _planner(s.spec)
    a.set_launch_mode(B.LAUNCH_GRAPH)
    b.set_launch_mode(B.LAUNCH_DIRECT)
    for pl in (a, b):
        _set_U(pl, s.U0)
    for _ in range(3):
        ra = H.gpu_replan(a, s.x0, s.obstacles)
        rb = H.gpu_replan(b, s.x0, s.obstacles)
        for k in ("S", "col", "label", "u_out", "U_new", "U_next"):
            assert np.array_equal(ra[k], rb[k]), k
        for k in ra["info"]:
            assert np.array_equal(np.asarray(ra["info"][k]), np.asarray(rb["info"][k])), k


def test_broad_phase_keeps_every_reachable_obstacle():
    """Rollouts at the speed bound reach max|v| N dt: an obstacle whose
    surface lies just inside that reach is hit, one just beyond the margin is
    left out, and every collision flag and first contact equals the oracle's
    (which tests every obstacle)."""
    import math

    N, dt, v = 40, 0.05, 0.8
    reach = v * N * dt
    spec = W.PlannerSpec(num_samples=1024, horizon=N, dt=dt, noise_chol=W.diag_chol([0.5, 1e-3], 2),
                         u_min=W.TABLE1_UMIN, u_max=W.TABLE1_UMAX, dbscan_eps=0.3,
                         dbscan_min_pts=10, goal=[5.0, 0.0, 0, 0, 0, 0], seed=9).rounded()
    R = 0.3
    # surfaces at reach - 0.01 (hit), reach + 0.0025 (inside the margin, no
    # contact) and reach + 0.02 (left out), on three headings fanned around +x
    obs = []
    for d, ang in ((reach - 0.01, 0.0), (reach + 0.0025, 0.6), (reach + 0.02, -0.6)):
        c = d + R
        obs.append([c * math.cos(ang), c * math.sin(ang), R])
    obs = np.asarray(obs, np.float32)
    U0 = np.zeros((N, 2), np.float32)
    U0[:, 0] = 5.0  # every step clamps at the bound
    x0 = np.zeros(3, np.float32)
    pl = _planner(spec)
    _set_U(pl, U0)
    r = H.gpu_replan(pl, x0, obs)
    o = oracle.replan(spec, x0, U0, obs)
    _compare_rollouts(r, o, spec)
    assert int(o["col"].sum()) > 0 and set(np.unique(o["first_obs"][o["col"] == 1])) == {0}
    assert np.array_equal(r["col"], o["col"])


def test_time_rollout_restores_state():
    """The rollout-only timing call leaves the planner exactly as it was."""
    s = W.unicycle_dynamic_ahead(4, num_samples=1024)
    pl = _planner(s.spec)
    _set_U(pl, s.U0)
    a0 = H.gpu_replan(pl, s.x0, s.obstacles)
    state = pl.get_state()
    a1 = H.gpu_replan(pl, s.x0, s.obstacles)
    pl.set_state(state)
    ms = pl.time_rollout(H.to_dev(s.x0), H.to_dev(s.obstacles), reps=5)
    assert ms > 0.0
    b1 = H.gpu_replan(pl, s.x0, s.obstacles)
    for k in ("S", "col", "u_out", "U_new", "U_next"):
        assert np.array_equal(a1[k], b1[k]), k
    assert a1["info"]["step"] == b1["info"]["step"] == a0["info"]["step"] + 1



def test_tune_launch_restores_state_and_picks_a_mode():
    """The launch-mode tuner leaves the planner as it was (the next replan
    equals the one it would have been) and keeps the faster mode; both modes
    give the same bits."""
    from paper_2607_06499_amd import binding as B

    s = W.unicycle_dynamic_ahead(6, num_samples=2048)
    pl = _planner(s.spec)
    _set_U(pl, s.U0)
    a0 = H.gpu_replan(pl, s.x0, s.obstacles)
    state = pl.get_state()
    a1 = H.gpu_replan(pl, s.x0, s.obstacles)
    pl.set_state(state)
    ug, ud = pl.tune_launch(H.to_dev(s.x0), H.to_dev(s.obstacles), reps=4)
    assert ug > 0.0 and ud > 0.0
    b1 = H.gpu_replan(pl, s.x0, s.obstacles)
    for k in ("S", "col", "u_out", "U_new", "U_next"):
        assert np.array_equal(a1[k], b1[k]), k
    assert a1["info"]["step"] == b1["info"]["step"] == a0["info"]["step"] + 1
    with pytest.raises(B.CeMppiError):
        pl.tune_launch(H.to_dev(s.x0), H.to_dev(s.obstacles), reps=0)

def _lockstep(scene, steps, tag, pl=None, on_step=None):
    """Closed loop in lockstep: at every step both sides start from the same
    state, nominal sequence and observation history (the loop follows the
    oracle's output); every rollout record and every later stage is
    compared.  Returns the per-step counts of _check_post."""
    spec = scene.spec
    pl = pl if pl is not None else _planner(spec)
    fld = scene.field.copy()
    x = scene.x0.astype(np.float64)
    U = scene.U0.astype(np.float64)
    hist = []
    out = []
    for t in range(steps):
        obs = fld.observation()
        hist.insert(0, obs[:, : spec.p].astype(np.float64))
        hist = hist[: spec.history_len]
        x32, U32, hs = np.float32(x), np.float32(U), np.array(hist)
        _set_U(pl, U32)
        r = H.gpu_replan(pl, x32, obs)
        o = oracle.replan(spec, x32, U32, obs, hs, step=t)
        assert r["info"]["step"] == t
        bnd = _compare_rollouts(r, o, spec)
        if on_step is not None:
            on_step(t, x32, U32, obs, hs, o)
        o, nflip = _resolve(spec, x32, U32, obs, hs, t, o, r, bnd)
        st = _check_post(r, o, spec, U32, obs, hist=hs, tag=f"{tag} t={t}")
        _check_output_shift(r["U_new"], r["u_out"], r["U_next"])
        st.update(boundary=int(bnd.sum()), resolved=nflip, o_rule=o["rule"], o_M=o["n_clusters"],
                  o_selected=o["selected"])
        out.append(st)
        U = o["U_next"]
        x = (oracle.unicycle_step(x, o["u_out"], spec.dt) if spec.dynamics == W.UNICYCLE
             else _arm_step(x, o["u_out"], spec.dt))
        fld.step(spec.dt)
    return out


def test_lockstep_dynamic_loop():
    """unicycle_dynamic shaped scene, eight closed-loop steps in lockstep
    (history included): every step is compared."""
    st = _lockstep(W.unicycle_dynamic_ahead(3, num_samples=2048), 8, "dynamic_ahead_2048")
    assert all(x["branch"] == 0 for x in st)


def _arm_ahead(seed=1, num_samples=4096):
    base = W.arm6_dynamic(seed, num_samples)
    org, _ = oracle.arm_frames(base.x0[:6].astype(np.float64), np.asarray(base.spec.dh, np.float64).reshape(6, 4))
    cen = oracle.arm_spheres(org, base.spec.n_link_spheres)
    return W.arm6_dynamic_ahead(cen[-1], seed, num_samples)


FULL = [
    ("unicycle_static", lambda: W.unicycle_static(1), False),
    ("unicycle_static_ahead", lambda: W.unicycle_static_ahead(1), True),
    ("unicycle_dynamic", lambda: W.unicycle_dynamic(1), False),
    ("unicycle_dynamic_ahead", lambda: W.unicycle_dynamic_ahead(1), True),
    ("arm6_dynamic", lambda: W.arm6_dynamic(1), False),
    ("arm6_dynamic_ahead", lambda: _arm_ahead(1), True),
]


@pytest.mark.parametrize("name,make,clusters", FULL, ids=[f[0] for f in FULL])
def test_full_size_workloads_match_oracle(name, make, clusters):
    """The benchmark's single-planner workloads at their full sizes (K up to
    8192, N up to 50) in the launch configuration the benchmark times (the
    library default), three closed-loop steps in lockstep with the oracle:
    every rollout record element by element, then every later stage.  The
    'ahead' scenes put an obstacle in the way so that every step takes the
    clustering branch; there DBSCAN runs on about 1,000 to 8,000 points and
    its labels are checked point by point."""
    s = make()
    st = _lockstep(s, 3, name)
    flagged = sum(x["boundary"] for x in st)
    print(f"{name}: K={s.spec.num_samples} N={s.spec.horizon}, {flagged} boundary rollouts flagged, "
          f"branches {[x['branch'] for x in st]}, V {[x.get('V') for x in st]}")
    assert flagged <= 3 * max(4, s.spec.num_samples // 1000)
    if clusters:
        assert all(x["branch"] == 0 for x in st), st
        assert sum(x["M"] >= 1 for x in st) >= 2, st


CROSSING = [
    ("left_2048", dict(side=1, num_samples=2048, distance=1.5, speed=0.5), 6),
    ("right_8192", dict(side=-1, num_samples=8192, distance=1.2, speed=0.5), 3),
    ("left_8192", dict(side=1, num_samples=8192, distance=1.5, speed=0.5), 5),
]


@pytest.mark.parametrize("name,kw,steps", CROSSING, ids=[c[0] for c in CROSSING])
def test_dynamic_rule_crossing_obstacle(name, kw, steps):
    """An obstacle crossing the robot's path (Sec. II-B.3): from the second
    observation on, the dynamic rule of Eq. (18) picks among two clusters.
    At every step the GPU's velocity estimate (Eq. (17)), rule, cluster
    directions and selection are compared with the oracle's; at least one
    step picks a different cluster than the static rule of Eq. (14) would."""
    s = W.unicycle_crossing(1, **kw)
    st = _lockstep(s, steps, name)
    dyn2 = [x for x in st if x.get("rule") == 1 and x.get("M", 0) >= 2]
    print(f"{name}: {len(dyn2)} steps with the dynamic rule over two or more clusters; "
          f"selected {[x.get('selected') for x in st]}")
    assert len(dyn2) >= 1
    assert all(not x.get("near_tie") for x in dyn2)


def test_dynamic_rule_differs_from_static_choice():
    """On the crossing scene the cluster of Eq. (18) is not the one of
    minimum mean cost at some step: the dynamic argmin is exercised, not a
    trivial one."""
    s = W.unicycle_crossing(1, side=1, num_samples=2048, distance=1.5, speed=0.5)
    differs = []

    def probe(t, x, U, obs, hist, o):
        if o["rule"] == 1 and o["n_clusters"] >= 2:
            differs.append(int(o["selected"]) != int(np.argmin(o["c_mean_cost"])))

    _lockstep(s, 6, "crossing_static_vs_dynamic", on_step=probe)
    assert any(differs), differs


def test_degenerate_branches():
    # every rollout collides
    s = W.unicycle_static_ahead(1)
    s.field.c[0] = s.x0[:2]
    s.field.r[0] = 5.0
    pl = _planner(s.spec)
    _set_U(pl, s.U0)
    r = H.gpu_replan(pl, s.x0, s.obstacles)
    o = oracle.replan(s.spec, s.x0, s.U0, s.obstacles)
    assert r["info"]["branch"] == 2 == o["branch"] and r["info"]["status"] == o["status"]
    _check_post(r, o, s.spec, s.U0, s.obstacles, tag="all_collide")
    # no cluster (minPts larger than |V|)
    s = W.unicycle_static_ahead(1)
    s.spec = s.spec.replace(dbscan_min_pts=100000)
    pl = _planner(s.spec)
    _set_U(pl, s.U0)
    r = H.gpu_replan(pl, s.x0, s.obstacles)
    o = oracle.replan(s.spec, s.x0, s.U0, s.obstacles)
    assert r["info"]["status"] == o["status"] and r["info"]["n_clusters"] == 0
    bnd = _compare_rollouts(r, o, s.spec)
    o, _ = _resolve(s.spec, s.x0, s.U0, s.obstacles, None, 0, o, r, bnd)
    st = _check_post(r, o, s.spec, s.U0, s.obstacles, tag="no_cluster")
    assert st["M"] == 0 and st.get("e2e_update"), st
    # non-finite input: no-op
    x = s.x0.copy()
    x[0] = np.nan
    before = pl.get_nominal().cpu().numpy()
    r = H.gpu_replan(pl, x, s.obstacles)
    assert r["info"]["status"] & 16
    assert np.array_equal(r["U_next"], before)
    assert np.array_equal(r["u_out"], before[0])


def test_tiny_problem():
    s = W.random_scene(21, num_samples=1, horizon=1, n_obs=1)
    pl = _planner(s.spec)
    _set_U(pl, s.U0)
    r = H.gpu_replan(pl, s.x0, s.obstacles)
    o = oracle.replan(s.spec, s.x0, s.U0, s.obstacles)
    assert r["info"]["branch"] == o["branch"]
    assert H.rel_err(r["S"], o["S"]).max() <= H.TRAJ_RTOL
    assert np.abs(r["U_new"] - o["U_new"]).max() <= 1e-5
    _check_post(r, o, s.spec, s.U0, s.obstacles, tag="tiny")


# ------------------------------------------------------------------ variants
VARIANT_ROLLOUTS = [
    ("arm_pose", lambda: _with_flags(W.random_scene(31, dynamics=W.ARM6, num_samples=700, horizon=20,
                                                    n_obs=10), W.FLAG_POSE_COST, rv=(0.3, -1.1, 0.6))),
    ("arm_pose_contact_at_start", lambda: _arm_touching_at_start()),
    ("arm6_pose", lambda: W.arm6_pose(2, num_samples=1500)),
]


def _with_flags(s, flags, rv=None):
    spec = s.spec.replace(flags=flags)
    if rv is not None:
        spec = spec.replace(goal=list(spec.goal[:3]) + list(rv), Q=[10.0, 3.0, 1000.0, 0, 0, 0],
                            Qf=[10.0, 3.0, 500.0, 0, 0, 0])
    return W.Scene(spec, s.x0, s.U0, s.field, s.name)


def _arm_touching_at_start():
    """Pose cost with an obstacle already touching the arm at x_0: every
    rollout pays w_c for the start state."""
    s = _with_flags(W.random_scene(32, dynamics=W.ARM6, num_samples=600, horizon=16, n_obs=6),
                    W.FLAG_POSE_COST, rv=(1.0, 0.2, -0.4))
    org, _ = oracle.arm_frames(s.x0[:6].astype(np.float64), np.asarray(s.spec.dh, np.float64).reshape(6, 4))
    cen = oracle.arm_spheres(org, s.spec.n_link_spheres)
    s.field.c[0] = cen[2] + np.array([0.0, 0.0, 0.03])
    s.field.r[0] = 0.06
    return s


@pytest.mark.parametrize("name,make", VARIANT_ROLLOUTS, ids=[v[0] for v in VARIANT_ROLLOUTS])
def test_pose_cost_rollouts_match_oracle(name, make):
    s = make()
    pl = _planner(s.spec)
    _set_U(pl, s.U0)
    r = H.gpu_replan(pl, s.x0, s.obstacles)
    o = oracle.replan(s.spec, s.x0, s.U0, s.obstacles)
    bnd = _compare_rollouts(r, o, s.spec)
    if name == "arm_pose_contact_at_start":
        assert np.all(o["S"] >= 1000.0) and np.all(r["S"] >= 1000.0)
    o, nflip = _resolve(s.spec, s.x0, s.U0, s.obstacles, None, 0, o, r, bnd)
    st = _check_post(r, o, s.spec, s.U0, s.obstacles, tag=name)
    print(f"{name}: {int(bnd.sum())} boundary rollouts, {nflip} resolved; {st}")
    assert int(bnd.sum()) <= 3


def _arm_step(x, u, dt):
    x = np.asarray(x, np.float64).copy()
    x[:6] = x[:6] + np.asarray(u, np.float64) * dt
    x[6:] = u
    return x


LOCKSTEP_CV = [
    ("random_uni_cv", lambda: _with_flags(W.random_scene(34, num_samples=1500, horizon=30, n_obs=8,
                                                          scene_mode=W.DYNAMIC), W.FLAG_OBS_CONST_VEL)),
    ("unicycle_dynamic_cv_ahead", lambda: _cv_ahead()),
    ("arm6_pose", lambda: W.arm6_pose(4, num_samples=1024)),
]


def _cv_ahead():
    s = W.unicycle_dynamic_ahead(2, num_samples=2048)
    return W.Scene(s.spec.replace(flags=W.FLAG_OBS_CONST_VEL), s.x0, s.U0, s.field, s.name)


@pytest.mark.parametrize("name,make", LOCKSTEP_CV, ids=[v[0] for v in LOCKSTEP_CV])
def test_constant_velocity_lockstep_loop(name, make):
    """Closed loop in lockstep with constant-velocity obstacles: both sides
    hold the same observation history, so every obstacle's velocity (and with
    it every contact) is predicted alike from the second step on."""
    s = make()
    spec = s.spec
    moved = []

    def frozen_differs(t, x, U, obs, hist, o):
        # the frozen model on the same inputs differs once velocities exist
        if t >= 1:
            fz = oracle.replan(spec.replace(flags=spec.flags & ~W.FLAG_OBS_CONST_VEL), x, U, obs, hist, step=t)
            moved.append(not np.array_equal(fz["col"], o["col"]))

    st = _lockstep(s, 6, name, on_step=frozen_differs)
    assert len(st) == 6
    assert any(moved)


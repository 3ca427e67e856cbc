"""Batched form: every member of a batch gets bitwise the result of its own
single-planner replan (same configuration, nominal, history and step), for
members of uneven size and of every kind (2-D members on the angular windows
and on the sorted distance passes, arms), over consecutive steps and under
every tuning the autotuner may pick; and every member matches the FP64
oracle's replan on its inputs, stage by stage."""
import numpy as np
import pytest

import oracle
from paper_2607_06499_amd import workloads as W
from tests import harness as H
from tests import test_gpu_parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not H.gpu_ok():
        pytest.skip("no GPU")


MEMBERS = [
    lambda: W.random_scene(21, num_samples=300, horizon=20, n_obs=5),
    lambda: W.random_scene(22, num_samples=1111, horizon=45, n_obs=12),
    lambda: W.unicycle_static_ahead(3, num_samples=700),
    lambda: W.unicycle_dynamic_ahead(2, num_samples=2048),
    lambda: W.random_scene(23, dynamics=W.ARM6, num_samples=400, horizon=16, n_obs=6),
    lambda: W.arm6_dynamic(4, num_samples=512),
    lambda: W.random_scene(24, num_samples=64, horizon=1, n_obs=0),
    lambda: W.paper_arm_preset(2),
    lambda: W.unicycle_dynamic_cv(5, num_samples=1024),
    lambda: W.arm6_pose(6, num_samples=640),
    # large enough for two rollout rounds per wave in the single-planner launch
    lambda: W.unicycle_dynamic_ahead(4, num_samples=8192),
]

TUNINGS = [None, (1, 2, 2, 1), (4, 16, 4, 8), (8, 4, 2, 2)]

# 2-D members put on the distance passes before the batch is made: the batch
# runs them on its spatially sorted passes, the other 2-D members on the
# angular windows
TILED = (1, 8)


def _setup():
    from paper_2607_06499_amd import binding as B

    scenes = [m() for m in MEMBERS]
    batched = [B.Planner(s.spec) for s in scenes]
    single = [B.Planner(s.spec) for s in scenes]
    for i, (s, a, b) in enumerate(zip(scenes, batched, single)):
        a.set_nominal(H.to_dev(s.U0))
        b.set_nominal(H.to_dev(s.U0))
        if i in TILED:
            a.set_dbscan_mode(B.DBSCAN_TILED)
            b.set_dbscan_mode(B.DBSCAN_TILED)
    paths = {a.dbscan_path() for a in batched}
    assert {B.DBSCAN_WINDOW, B.DBSCAN_TILED, B.DBSCAN_BITMAP} <= paths  # 2-D both ways, and the arm
    xs = [H.to_dev(np.asarray(s.x0, np.float32)) for s in scenes]
    obs = [H.to_dev(np.asarray(s.obstacles, np.float32)) if len(s.obstacles) else None for s in scenes]
    batch = B.Batch(batched)
    batch.set_io(xs, obs)
    return B, scenes, batched, single, xs, obs, batch


def _compare(B, batched, single, tag):
    torch = H.torch_mod()
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(batched, single)):
        ia, ib = a.info(), b.info()
        for k in ia:
            assert np.array_equal(np.asarray(ia[k]), np.asarray(ib[k])), (tag, i, k)
        assert torch.equal(a.u_out, b.u_out), (tag, i)
        assert torch.equal(a.U_out, b.U_out), (tag, i)
        assert torch.equal(a.get_nominal(), b.get_nominal()), (tag, i)
        assert torch.equal(a.debug(B.DBG_COST, a.K), b.debug(B.DBG_COST, b.K)), (tag, i)
        if ia["branch"] == 0 and ia["n_feasible"] > 0:
            V = ia["n_feasible"]
            assert torch.equal(a.debug(B.DBG_LABEL, V), b.debug(B.DBG_LABEL, V)), (tag, i)


def test_batch_matches_single_replans_and_oracle():
    B, scenes, batched, single, xs, obs, batch = _setup()
    host_obs = [np.asarray(sc.obstacles, np.float32).copy() for sc in scenes]
    hists = [[] for _ in scenes]
    Us = [np.asarray(sc.U0, np.float64) for sc in scenes]
    kinds = set()
    summary = []
    for step, tune in enumerate(TUNINGS):
        if tune is not None:
            batch.set_tuning(*tune)
        # every step starts from the oracle's nominal (both forms get it)
        for i, (sc, a, b) in enumerate(zip(scenes, batched, single)):
            U32 = np.float32(Us[i])
            a.set_nominal(H.to_dev(U32))
            b.set_nominal(H.to_dev(U32))
            hists[i].insert(0, host_obs[i][:, : sc.spec.p].astype(np.float64))
            hists[i] = hists[i][: sc.spec.history_len]
        batch.replan()
        for b, x, o in zip(single, xs, obs):
            b.replan(x, o)
        _compare(B, batched, single, f"step {step} tuning {tune}")
        # each member against the oracle on the same inputs
        for i, (sc, a) in enumerate(zip(scenes, batched)):
            spec = sc.spec
            U32 = np.float32(Us[i])
            hs = np.array(hists[i]) if len(host_obs[i]) else None
            r = H.collect_outputs(a)
            o = oracle.replan(spec, sc.x0, U32, host_obs[i], hs, step=step)
            bnd = P._compare_rollouts(r, o, spec)
            o, nflip = P._resolve(spec, sc.x0, U32, host_obs[i], hs, step, o, r, bnd)
            st = P._check_post(r, o, spec, U32, host_obs[i], hist=hs, tag=f"member {i} step {step}")
            summary.append((i, step, st["branch"], st.get("V"), st.get("M")))
            Us[i] = o["U_next"]
        kinds |= {a.info()["branch"] for a in batched}
        # the obstacles move between steps (in place: both forms read the same
        # tensors), so the constant-velocity members predict real motion
        H.torch_mod().cuda.synchronize()
        for o, ho in zip(obs, host_obs):
            if o is not None:
                o[:, 0] += 0.02
                o[:, 1] -= 0.01
                ho[:, 0] += np.float32(0.02)
                ho[:, 1] -= np.float32(0.01)
        H.torch_mod().cuda.synchronize()
        for o, ho in zip(obs, host_obs):
            if o is not None:
                assert np.array_equal(o.cpu().numpy(), ho)
    print("member, step, branch, V, M:", summary)
    # the members exercised the clustering branch and a fallback branch
    assert 0 in kinds and len(kinds) >= 2
    assert sum(1 for x in summary if x[2] == 0) >= 8
    batch.close()


def test_autotune_restores_state_and_keeps_results():
    B, scenes, batched, single, xs, obs, batch = _setup()
    best, ms = batch.autotune(reps=2)
    assert best["colg"] in (2, 4, 8) and ms > 0.0
    assert batch.get_tuning() == best
    # the tuner left every member where it was: the next batch replan is the
    # first step of each member
    batch.replan()
    for b, x, o in zip(single, xs, obs):
        b.replan(x, o)
    _compare(B, batched, single, f"after autotune {best}")
    assert all(a.info()["step"] == 0 for a in batched)
    batch.close()


def test_subset_launches_match_single_replans():
    """Launches over member subsets (the continuous-batching primitive), on
    two streams, give each listed member exactly its single-planner step."""
    B, scenes, batched, single, xs, obs, batch = _setup()
    torch = H.torch_mod()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    rounds = [[0, 2, 4, 6, 8, 10], [1, 3, 5, 7, 9], [7, 0], [9, 2, 3, 4], [5, 8, 10], [6, 1, 0], [8, 9]]
    for i, members in enumerate(rounds):
        with torch.cuda.stream(streams[i % 2]):
            batch.replan_subset(members, stream=streams[i % 2])
        streams[i % 2].synchronize()
        for m in members:
            single[m].replan(xs[m], obs[m])
        torch.cuda.synchronize()
        for m in members:
            assert torch.equal(batched[m].u_out, single[m].u_out), (i, m)
            assert torch.equal(batched[m].get_nominal(), single[m].get_nominal()), (i, m)
            ia, ib = batched[m].info(), single[m].info()
            for k in ia:
                assert np.array_equal(np.asarray(ia[k]), np.asarray(ib[k])), (i, m, k)
    with pytest.raises(B.CeMppiError):
        batch.replan_subset([0, 0])
    with pytest.raises(B.CeMppiError):
        batch.replan_subset([len(batched)])
    batch.close()


def test_batch_rejects_bad_io():
    from paper_2607_06499_amd import binding as B

    s = W.random_scene(25, num_samples=128, horizon=10, n_obs=3)
    pl = B.Planner(s.spec)
    batch = B.Batch([pl])
    batch.set_io([H.to_dev(np.asarray(s.x0, np.float32))], [H.to_dev(np.asarray(s.obstacles, np.float32))])
    batch._io[0].n_obs = 65
    with pytest.raises(B.CeMppiError):
        batch.replan()
    batch._io[0].n_obs = 3
    batch._io[0].u_out = None
    with pytest.raises(B.CeMppiError):
        batch.replan()
    with pytest.raises(B.CeMppiError):
        B.Batch([pl, pl])
    batch.close()


def test_batch_large_window_members_match_single():
    """Members of up to 16,384 rollouts on the angular windows (many
    count-and-place items per member, zones that may leave LDS) replan in a
    batch bitwise as they do alone, over three closed-loop steps."""
    from paper_2607_06499_amd import binding as B
    from paper_2607_06499_amd.plant import unicycle_step

    scenes = [W.unicycle_dynamic_ahead(1, num_samples=16384), W.unicycle_dynamic_ahead(3, num_samples=12000),
              W.unicycle_static_ahead(3, num_samples=4096)]
    batched = [B.Planner(s.spec) for s in scenes]
    single = [B.Planner(s.spec) for s in scenes]
    for s, a, b in zip(scenes, batched, single):
        a.set_nominal(H.to_dev(s.U0))
        b.set_nominal(H.to_dev(s.U0))
        assert a.dbscan_path() == B.DBSCAN_WINDOW
    fields = [s.field.copy() for s in scenes]
    xs = [s.x0.astype(np.float64) for s in scenes]
    batch = B.Batch(batched)
    clustered = 0
    for step in range(3):
        xd = [H.to_dev(np.float32(x)) for x in xs]
        od = [H.to_dev(np.asarray(f.observation(), np.float32)) for f in fields]
        batch.set_io(xd, od)
        batch.replan()
        for b, x, o in zip(single, xd, od):
            b.replan(x, o)
        _compare(B, batched, single, f"large step {step}")
        for i, a in enumerate(batched):
            info = a.info()
            clustered += info["branch"] == 0 and info["n_clusters"] >= 1
            xs[i] = unicycle_step(xs[i], a.u_out.cpu().numpy(), scenes[i].spec.dt)
            fields[i].step(scenes[i].spec.dt)
    assert clustered >= 2
    batch.close()

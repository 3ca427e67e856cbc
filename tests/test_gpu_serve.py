"""Served form: continuous batching over resident sessions.  Each request's
result equals, bitwise, the result of replanning its session alone with the
same sequence of requests, and matches the FP64 oracle stage by stage;
admission is bounded by device memory; the plain form launches one request
at a time."""
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


def _scenes():
    out = []
    for i in range(12):
        if i % 3 == 2:
            s = W.random_scene(40 + i, dynamics=W.ARM6, num_samples=256 + 37 * i, horizon=12 + i,
                               n_obs=4 + i % 5)
        else:
            s = W.random_scene(40 + i, num_samples=300 + 101 * i, horizon=15 + 3 * i, n_obs=3 + i)
        s.spec = s.spec.replace(stream_id=i)
        out.append(s)
    return out


def _trace(scenes, n, rate, seed=3):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    sess = rng.integers(0, len(scenes), size=n).astype(np.int32)
    x = np.zeros((n, 12), np.float32)
    ob = np.zeros((n, 256), np.float32)
    no = np.zeros(n, np.int32)
    for i, s in enumerate(sess):
        sc = scenes[s]
        x[i, : len(sc.x0)] = sc.x0
        o = np.asarray(sc.obstacles, np.float32)
        no[i] = len(o)
        ob[i, : o.size] = o.ravel()
    return t, sess, x, ob, no


def test_mixed_results_equal_alone():
    from paper_2607_06499_amd import binding as B

    scenes = _scenes()
    srv = B.Server(max_batch=8, max_inflight=3)
    for s in scenes:
        srv.open_session(s.spec, s.U0)
    srv.start()
    t, sess, x, ob, no = _trace(scenes, 150, rate=50_000.0)
    lat, u = srv.run_trace(t, sess, x, ob, no)
    st = srv.stats()
    srv.close()
    assert st["served"] == 150 and st["mean_batch"] > 1.0, st
    assert np.all(lat > 0.0)
    # every session alone, with the same sequence of requests
    torch = H.torch_mod()
    for k, sc in enumerate(scenes):
        pl = B.Planner(sc.spec)
        pl.set_nominal(H.to_dev(sc.U0))
        xd = H.to_dev(np.asarray(sc.x0, np.float32))
        od = H.to_dev(np.asarray(sc.obstacles, np.float32))
        m = pl.m
        for i in np.flatnonzero(sess == k):
            uu, _, _ = pl.replan(xd, od)
            torch.cuda.synchronize()
            assert np.array_equal(uu.cpu().numpy(), u[i, :m]), (k, int(i))
        pl.close()


def test_served_requests_match_oracle():
    """Rounds of one request per session, submitted together so that they
    share launches; before each round every session's nominal is set to the
    oracle's (lockstep).  Each request is compared with the oracle's replan
    of its session through every stage (the session planner's buffers hold
    that request's replan)."""
    from paper_2607_06499_amd import binding as B

    scenes = _scenes()[:9]
    srv = B.Server(max_batch=16, max_inflight=3)
    for s in scenes:
        srv.open_session(s.spec, s.U0)
    srv.start()
    views = [srv.session_planner(i, s.spec) for i, s in enumerate(scenes)]
    Us = [np.asarray(s.U0, np.float64) for s in scenes]
    hists = [[] for _ in scenes]
    torch = H.torch_mod()
    branches = []
    for rnd in range(3):
        for i, (sc, v) in enumerate(zip(scenes, views)):
            v.set_nominal(H.to_dev(np.float32(Us[i])))
            hists[i].insert(0, np.asarray(sc.obstacles, np.float64)[:, : sc.spec.p])
            hists[i] = hists[i][: sc.spec.history_len]
        torch.cuda.synchronize()
        tickets = [srv.submit(i, sc.x0, sc.obstacles) for i, sc in enumerate(scenes)]
        res = [srv.wait(t, i) for i, t in enumerate(tickets)]
        for i, (sc, v) in enumerate(zip(scenes, views)):
            u, info, lat = res[i]
            assert info["step"] == rnd and lat > 0.0
            spec = sc.spec
            U32 = np.float32(Us[i])
            hs = np.array(hists[i])
            r = H.collect_outputs(v, info=info, u_out=u[: spec.m])
            o = oracle.replan(spec, sc.x0, U32, sc.obstacles, hs, step=rnd)
            bnd = P._compare_rollouts(r, o, spec)
            o, _ = P._resolve(spec, sc.x0, U32, sc.obstacles, hs, rnd, o, r, bnd)
            st = P._check_post(r, o, spec, U32, sc.obstacles, hist=hs, tag=f"session {i} request {rnd}")
            branches.append(st["branch"])
            Us[i] = o["U_next"]
    stats = srv.stats()
    srv.close()
    assert stats["served"] == 3 * len(scenes) and stats["mean_batch"] > 1.0, stats
    assert 0 in branches, branches


def test_admission_bounded_by_memory():
    from paper_2607_06499_amd import binding as B

    scenes = _scenes()[:3]
    probe = B.Server(max_batch=4, max_inflight=1)
    probe.open_session(scenes[0].spec)
    one = probe.stats()["session_bytes"]
    probe.close()
    srv = B.Server(max_batch=4, max_inflight=1, memory_budget=one)
    srv.open_session(scenes[0].spec)
    with pytest.raises(B.CeMppiError) as e:
        srv.open_session(scenes[0].spec)
    assert e.value.status == B.CE_EBUSY
    srv.close()


def test_plain_form_is_one_request_per_launch():
    """The plain served form: one request at a time through ce_mppi_replan of
    its session (single-planner kernels), bitwise equal to replanning the
    session alone; the batched server with max_batch = 1 also launches one
    request at a time."""
    from paper_2607_06499_amd import binding as B

    scenes = _scenes()[:4]
    with pytest.raises(B.CeMppiError):
        B.Server(max_batch=4, max_inflight=1, mode=B.SERVE_PLAIN)
    srv = B.Server(max_batch=1, max_inflight=1, mode=B.SERVE_PLAIN)
    for s in scenes:
        srv.open_session(s.spec, s.U0)
    srv.start()
    t, sess, x, ob, no = _trace(scenes, 40, rate=20_000.0, seed=5)
    lat, u = srv.run_trace(t, sess, x, ob, no)
    st = srv.stats()
    srv.close()
    assert st["launches"] == 40 and st["mean_batch"] == 1.0 and st["max_inflight"] == 1
    torch = H.torch_mod()
    for k, sc in enumerate(scenes):
        pl = B.Planner(sc.spec)
        pl.set_nominal(H.to_dev(sc.U0))
        xd = H.to_dev(np.asarray(sc.x0, np.float32))
        od = H.to_dev(np.asarray(sc.obstacles, np.float32))
        for i in np.flatnonzero(sess == k):
            uu, _, _ = pl.replan(xd, od)
            torch.cuda.synchronize()
            assert np.array_equal(uu.cpu().numpy(), u[i, : pl.m]), (k, int(i))
        pl.close()
    srv = B.Server(max_batch=1, max_inflight=1)
    for s in scenes:
        srv.open_session(s.spec, s.U0)
    srv.start()
    lat, u = srv.run_trace(t, sess, x, ob, no)
    st = srv.stats()
    srv.close()
    assert st["launches"] == 40 and st["mean_batch"] == 1.0 and st["max_inflight"] == 1

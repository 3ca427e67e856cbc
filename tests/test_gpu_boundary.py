"""Boundary calls on the GPU: the obstacle history set through the C-ABI
behaves exactly like the history a planner builds from its own replans, and
a replan on a second stream while the first still has work queued is
refused with CE_EBUSY."""
import numpy as np
import pytest

from paper_2607_06499_amd import workloads as W
from tests import harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not H.gpu_ok():
        pytest.skip("no GPU")


def test_set_history_equals_pushed_history():
    """Planner A replans steps 0..3 of a dynamic scene; planner B gets A's
    nominal and step before step 3 and the three earlier observations through
    set_history: its step-3 replan is bitwise A's (velocity estimate and
    selection included).  More entries than history_len keep the newest."""
    from paper_2607_06499_amd import binding as B

    s = W.unicycle_crossing(1, side=1, num_samples=2048)
    spec = s.spec.replace(history_len=3)
    a, b = B.Planner(spec), B.Planner(spec)
    a.set_nominal(H.to_dev(s.U0))
    fld = s.field.copy()
    obs = []
    for t in range(4):
        obs.append(fld.observation())
        fld.step(spec.dt)
    x = H.to_dev(np.asarray(s.x0, np.float32))
    torch = H.torch_mod()
    for t in range(3):
        a.replan(x, H.to_dev(obs[t]))
    torch.cuda.synchronize()
    b.set_nominal(a.get_nominal())
    b.set_step(3)
    # five entries, newest first: only the newest two (history_len - 1 before
    # the push of step 3) matter once step 3 pushes its own observation
    stale = np.asarray(obs[0], np.float32).copy()
    stale[:, :2] += 7.0
    hist = np.stack([obs[2][:, :2], obs[1][:, :2], obs[0][:, :2], stale[:, :2], stale[:, :2]]).astype(np.float32)
    b.set_history(H.to_dev(hist))
    ra = H.gpu_replan(a, s.x0, obs[3])
    rb = H.gpu_replan(b, s.x0, obs[3])
    for k in ("u_out", "U_new", "U_next", "S", "label"):
        assert np.array_equal(ra[k], rb[k]), k
    for k in ra["info"]:
        assert np.array_equal(np.asarray(ra["info"][k]), np.asarray(rb["info"][k])), k
    assert ra["info"]["history_used"] == 3 and ra["info"]["rule"] == 1
    # an empty history: the dynamic rule cannot apply at the next replan
    b.set_history(H.to_dev(np.zeros((0, 1, 2), np.float32)))
    rc = H.gpu_replan(b, s.x0, obs[3])
    assert rc["info"]["status"] & B.STATUS_DYN_STATIC or rc["info"]["branch"] != 0
    with pytest.raises(B.CeMppiError):
        b.set_history(H.to_dev(np.zeros((2, 70, 2), np.float32)))
    a.close()
    b.close()


def test_replan_on_a_second_stream_while_busy():
    from paper_2607_06499_amd import binding as B

    torch = H.torch_mod()
    s = W.random_scene(3, num_samples=512, horizon=20, n_obs=4)
    pl = B.Planner(s.spec)
    pl.set_nominal(H.to_dev(s.U0))
    x = H.to_dev(np.asarray(s.x0, np.float32))
    o = H.to_dev(np.asarray(s.obstacles, np.float32))
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(sa):
        torch.cuda._sleep(100_000_000)  # bounded busy wait on stream a
        pl.replan(x, o, stream=sa)
    with pytest.raises(B.CeMppiError) as e:
        pl.replan(x, o, stream=sb)
    assert e.value.status == B.CE_EBUSY
    sa.synchronize()
    pl.replan(x, o, stream=sb)  # the previous stream is idle now
    sb.synchronize()
    assert pl.info()["step"] == 1
    # the same stream orders the calls itself
    with torch.cuda.stream(sb):
        torch.cuda._sleep(10_000_000)
        pl.replan(x, o, stream=sb)
        pl.replan(x, o, stream=sb)
    sb.synchronize()
    assert pl.info()["step"] == 3
    pl.close()

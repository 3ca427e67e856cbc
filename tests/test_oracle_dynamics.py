"""Pins of the oracle's forward simulation and cost (Eq. (4)-(5), Sec. III)
against closed forms."""
import math

import numpy as np
import pytest

from paper_2607_06499_amd import workloads as W


def _uni_spec(N=20, dt=0.1, **kw):
    base = dict(dynamics=W.UNICYCLE, horizon=N, num_samples=1, dt=dt,
                Q=[1.0, 2.0, 0.5, 0, 0, 0], R=[0.1, 0.3, 0, 0, 0, 0], Qf=[3.0, 4.0, 0.25, 0, 0, 0],
                goal=[2.0, -1.0, 0.5, 0, 0, 0])
    base.update(kw)
    return W.PlannerSpec(**base).rounded()


def test_straight_line_closed_form(orc):
    N, dt, v, th = 25, 0.1, 0.7, 0.3
    spec = _uni_spec(N, dt)
    dt = spec.dt
    x0 = np.array([0.2, -0.4, th])
    ut = np.tile([v, 0.0], (N, 1))
    r = orc.simulate(spec, x0, ut, np.zeros((0, 3)))
    j = np.arange(N + 1)
    exp = np.stack([x0[0] + v * j * dt * math.cos(th), x0[1] + v * j * dt * math.sin(th),
                    np.full(N + 1, th)], 1)
    assert np.allclose(r["traj"], exp, rtol=0, atol=1e-12)
    # cost: stage terms on x_0..x_{N-1} with the control term, terminal on x_N
    Q, R, Qf, g = (np.array(spec.Q[:3]), np.array(spec.R[:2]), np.array(spec.Qf[:3]),
                   np.array(spec.goal[:3]))
    S = sum(np.sum(Q * (exp[k] - g) ** 2) for k in range(N)) + N * np.sum(R * np.array([v, 0]) ** 2)
    S += np.sum(Qf * (exp[N] - g) ** 2)
    assert r["S"] == pytest.approx(S, rel=1e-12)
    assert r["col"] == 0 and r["first_obs"] == -1
    assert np.allclose(r["p_term"], exp[N, :2])


def test_constant_turn_chord_closed_form(orc):
    # explicit Euler with constant (v, w): the points lie on a circle of radius
    # v dt / (2 sin(w dt / 2)) and x_N - x_0 = v dt sin(N w dt/2)/sin(w dt/2) (cos, sin)(th0 + (N-1) w dt/2)
    N, dt, v, w, th0 = 30, 0.05, 0.9, 1.7, -0.4
    spec = _uni_spec(N, dt)
    dt = spec.dt
    r = orc.simulate(spec, np.array([1.0, 2.0, th0]), np.tile([v, w], (N, 1)), np.zeros((0, 3)))
    tr = r["traj"]
    chord = v * dt * math.sin(N * w * dt / 2) / math.sin(w * dt / 2)
    ang = th0 + (N - 1) * w * dt / 2
    assert np.allclose(tr[N, :2] - tr[0, :2], chord * np.array([math.cos(ang), math.sin(ang)]),
                       atol=1e-12)
    assert tr[N, 2] == pytest.approx(th0 + N * w * dt, abs=1e-12)
    rad = v * dt / (2 * math.sin(w * dt / 2))
    # centre: perpendicular bisector construction from the first two steps
    ctr = tr[0, :2] + rad * np.array([math.cos(th0 - w * dt / 2 + math.pi / 2),
                                      math.sin(th0 - w * dt / 2 + math.pi / 2)])
    ctr = ctr + rad * 0.0
    d = np.linalg.norm(tr[:, :2] - ctr, axis=1)
    # all points equidistant from the centre
    assert np.ptp(d) < 1e-10
    assert d[0] == pytest.approx(rad, rel=1e-10)


def test_unicycle_step_matches_paper_equations(orc):
    x = np.array([0.3, -0.2, 1.1])
    u = np.array([0.4, -2.0])
    dt = 0.07
    xn = orc.unicycle_step(x, u, dt)
    assert np.allclose(xn, [0.3 + 0.4 * math.cos(1.1) * dt, -0.2 + 0.4 * math.sin(1.1) * dt,
                            1.1 - 2.0 * dt], atol=1e-15)


def _dh(lengths):
    return np.array(W.arm_dh(lengths)).reshape(6, 4)


LEN = [0.16, 0.42, 0.39, 0.13, 0.10, 0.09]


def test_arm_fk_zero_pose_closed_form(orc):
    d1, a2, a3, d4, d5, d6 = LEN
    org, rot = orc.arm_frames(np.zeros(6), _dh(LEN))
    exp = np.array([[0, 0, 0], [0, 0, d1], [-a2, 0, d1], [-a2 - a3, 0, d1], [-a2 - a3, -d4, d1],
                    [-a2 - a3, -d4, d1 - d5], [-a2 - a3, -d4 - d6, d1 - d5]])
    assert np.allclose(org, exp, atol=1e-12)
    # end-effector frame at q = 0: R = Rx(pi/2) Rx(pi/2) Rx(-pi/2) = Rx(pi/2)
    assert np.allclose(rot, [[1, 0, 0], [0, 0, -1], [0, 1, 0]], atol=1e-12)


def test_arm_fk_base_rotation_and_wrist_invariance(orc):
    rng = np.random.default_rng(2)
    q = rng.uniform(-2, 2, 6)
    org, rot = orc.arm_frames(q, _dh(LEN))
    assert np.linalg.det(rot) == pytest.approx(1.0, abs=1e-12)
    assert np.allclose(rot @ rot.T, np.eye(3), atol=1e-12)
    # rotating joint 1 rotates every origin about the base z axis
    phi = 0.77
    q2 = q.copy()
    q2[0] += phi
    org2, _ = orc.arm_frames(q2, _dh(LEN))
    Rz = np.array([[math.cos(phi), -math.sin(phi), 0], [math.sin(phi), math.cos(phi), 0], [0, 0, 1]])
    assert np.allclose(org2, org @ Rz.T, atol=1e-12)
    # the last joint turns about its own axis: no origin moves
    q3 = q.copy()
    q3[5] += 1.3
    org3, _ = orc.arm_frames(q3, _dh(LEN))
    assert np.allclose(org3, org, atol=1e-12)
    # segment lengths sqrt(a^2 + d^2) do not depend on q
    seg = np.linalg.norm(np.diff(org, axis=0), axis=1)
    dh = _dh(LEN)
    assert np.allclose(seg, np.hypot(dh[:, 0], dh[:, 1]), atol=1e-12)


def test_arm_spheres_on_polyline(orc):
    rng = np.random.default_rng(5)
    org, _ = orc.arm_frames(rng.uniform(-1, 1, 6), _dh(LEN))
    ns = 8
    c = orc.arm_spheres(org, ns)
    seg = np.linalg.norm(np.diff(org, axis=0), axis=1)
    cum = np.concatenate([[0], np.cumsum(seg)])
    total = cum[-1]
    for s in range(ns):
        t = (s + 0.5) / ns * total
        i = min(np.searchsorted(cum, t, side="left") - 1, 5)
        i = max(i, 0)
        exp = org[i] + (t - cum[i]) / seg[i] * (org[i + 1] - org[i])
        assert np.allclose(c[s], exp, atol=1e-12)


def test_arm_integration_and_costs(orc):
    N, dt = 12, 0.05
    rng = np.random.default_rng(8)
    spec = W.PlannerSpec(dynamics=W.ARM6, horizon=N, num_samples=1, dt=dt, dh=list(_dh(LEN).ravel()),
                         goal=[0.3, -0.2, 0.5, 0, 0, 0], Q=[2.0, 0, 0, 0, 0, 0],
                         R=[0.1] * 6, Qf=[5.0, 0, 0, 0, 0, 0], q_limit=[0.2] * 6,
                         w_limit=10.0).rounded()
    dt = spec.dt
    q0 = rng.uniform(-0.3, 0.3, 6)
    ut = rng.uniform(-1, 1, (N, 6))
    r = orc.simulate(spec, np.concatenate([q0, np.zeros(6)]), ut, np.zeros((0, 4)))
    tr = r["traj"]
    assert np.allclose(tr[:, :6], q0 + dt * np.concatenate([np.zeros((1, 6)), np.cumsum(ut, 0)]),
                       atol=1e-12)
    assert np.allclose(tr[1:, 6:], ut, atol=0)
    dh = np.asarray(spec.dh).reshape(6, 4)
    goal = np.asarray(spec.goal[:3])
    qlim, wl = np.asarray(spec.q_limit), spec.w_limit

    def lim(q):
        e = np.maximum(np.abs(q) - qlim, 0.0)
        return wl * np.sum(e * e)

    S = 0.0
    for j in range(N):
        org, _ = orc.arm_frames(tr[j, :6], dh)
        S += spec.Q[0] * np.sum((org[6] - goal) ** 2) + lim(tr[j, :6]) + np.sum(np.asarray(spec.R) * ut[j] ** 2)
    org, _ = orc.arm_frames(tr[N, :6], dh)
    S += spec.Qf[0] * np.sum((org[6] - goal) ** 2) + lim(tr[N, :6])
    assert r["S"] == pytest.approx(S, rel=1e-12)
    assert np.allclose(r["p_term"], org[6])
    # the joint-limit penalty is active for this draw (|q| exceeds 0.2 somewhere)
    assert max(lim(tr[j, :6]) for j in range(N + 1)) > 0

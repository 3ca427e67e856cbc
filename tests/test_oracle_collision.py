"""Pins of the collision indicator, first contact and closest obstacle
(Sec. II-B.1, Sec. II-B.2) on hand-built geometry."""
import numpy as np

from paper_2607_06499_amd import workloads as W


def _spec(N=20, dt=0.1, robot_radius=0.0):
    return W.PlannerSpec(dynamics=W.UNICYCLE, horizon=N, num_samples=1, dt=dt,
                         robot_radius=robot_radius).rounded()


def _run(orc, obs, N=20, robot_radius=0.0, x0=(0.0, 0.0, 0.0), v=1.0, dt=0.1):
    spec = _spec(N, dt, robot_radius)
    return orc.simulate(spec, np.array(x0), np.tile([v, 0.0], (N, 1)),
                        np.asarray(obs, np.float32).reshape(-1, 3))


def test_first_contact_step_and_lowest_index(orc):
    # robot on the x axis at 0.1 m per step; obstacle A (index 1) is first
    # touched at x = 0.9 (j = 9); obstacle B (index 0) is touched at the same step
    A = (1.05, 0.0, 0.2)
    B = (1.2, 0.1, 0.35)
    r = _run(orc, [B, A])
    assert r["col"] == 1 and r["first_obs"] == 0
    assert np.allclose(r["p_first"], [0.9, 0.0], atol=1e-6)
    r = _run(orc, [A])
    assert r["col"] == 1 and r["first_obs"] == 0
    assert np.allclose(r["p_first"], [0.9, 0.0], atol=1e-6)
    # a later, lower-index obstacle does not change the first contact
    r = _run(orc, [(1.9, 0.0, 0.2), A])
    assert r["first_obs"] == 1


def test_outside_tangent_inside(orc):
    assert _run(orc, [(0.5, 0.5, 0.3)])["col"] == 0            # min distance 0.5 > 0.3
    # tangent at x_4 = 0.5 (dt = 1/8: every position and radius is exact):
    # distance equals the radius -> contact (closed ball); a radius one ulp
    # smaller leaves the rollout free
    r = _run(orc, [(0.5, 0.25, 0.25)], N=8, dt=0.125)
    assert r["col"] == 1 and np.allclose(r["p_first"], [0.5, 0.0], atol=0.0)
    r = _run(orc, [(0.5, 0.25, float(np.nextafter(np.float32(0.25), np.float32(0))))], N=8, dt=0.125)
    assert r["col"] == 0
    # robot radius adds to the obstacle radius
    assert _run(orc, [(0.5, 0.5, 0.3)], robot_radius=0.25)["col"] == 1
    # the start state is not checked; the first state after it is
    r = _run(orc, [(0.0, 0.0, 0.15)], v=1.0)
    assert r["col"] == 1 and np.allclose(r["p_first"], [0.1, 0.0], atol=1e-6)
    r = _run(orc, [(0.0, 0.0, 0.05)], v=1.0)
    assert r["col"] == 0


def test_boundary_clearance(orc):
    # relative distance to the nearest contact boundary over the trajectory
    r = _run(orc, [(0.5, 0.5, 0.3)], N=10)
    assert abs(r["clearance"] - (0.5 - 0.3) / 0.3) < 1e-6


def test_closest_obstacle_ties_to_lowest_index(orc):
    spec = _spec()
    x0 = np.array([0.0, 0.0, 0.0])
    obs = np.array([(-3.0, 0.0, 0.1), (1.0, 0.0, 0.5), (0.0, 2.0, 1.5), (0.0, -4, 0.2)], np.float32)
    assert orc.closest_obstacle(spec, x0, obs) == 1          # clearances 2.9, 0.5, 0.5, 3.8
    obs2 = obs[[0, 3, 2, 1]]
    assert orc.closest_obstacle(spec, x0, obs2) == 2
    assert orc.closest_obstacle(spec, x0, np.zeros((0, 3), np.float32)) == -1


def test_arm_collision_against_link_spheres(orc):
    lengths = [0.16, 0.42, 0.39, 0.13, 0.10, 0.09]
    spec = W.PlannerSpec(dynamics=W.ARM6, horizon=4, num_samples=1, dt=0.05,
                         dh=W.arm_dh(lengths), n_link_spheres=8, link_sphere_radius=0.05).rounded()
    dh = np.asarray(spec.dh).reshape(6, 4)
    org, _ = orc.arm_frames(np.zeros(6), dh)
    cen = orc.arm_spheres(org, 8)
    x0 = np.zeros(12)
    ut = np.zeros((4, 6))
    # an obstacle touching sphere 3 at q = 0 (held still): contact at j = 1
    o = cen[3] + np.array([0.0, 0.0, 0.05 + 0.07 - 1e-3])
    r = orc.simulate(spec, x0, ut, np.array([[5, 5, 5, 0.1], [*o, 0.07]], np.float32))
    assert r["col"] == 1 and r["first_obs"] == 1
    o = cen[3] + np.array([0.0, 0.0, 0.05 + 0.07 + 1e-3])
    r = orc.simulate(spec, x0, ut, np.array([[*o, 0.07]], np.float32))
    assert r["col"] == 0


def test_closest_obstacle_margin(orc):
    spec = _spec()
    x0 = np.array([0.0, 0.0, 0.0])
    # clearances 2.9, 0.5, 0.75, 3.8: o* = 1, margin 0.25
    obs = np.array([(-3.0, 0.0, 0.1), (1.0, 0.0, 0.5), (0.0, 2.0, 1.25), (0.0, -4, 0.2)], np.float32)
    i, mg = orc.closest_obstacle_margin(spec, x0, obs)
    assert i == 1 and abs(mg - 0.25) < 1e-7
    # an exact tie: margin 0, lowest index
    obs = np.array([(0.0, 2.0, 1.5), (1.0, 0.0, 0.5)], np.float32)
    i, mg = orc.closest_obstacle_margin(spec, x0, obs)
    assert i == 0 and mg == 0.0
    i, mg = orc.closest_obstacle_margin(spec, x0, obs[:1])
    assert i == 0 and mg == np.inf


def test_contact_decided_in_double_precision(orc):
    # positions j/8 and the radii are exact: a gap of 1e-12 m separates contact
    # from no contact (single precision would call both a contact)
    spec = _spec(8, 0.125)
    ut = np.tile([1.0, 0.0], (8, 1))
    for dy, col in ((1e-12, 0), (-1e-12, 1), (0.0, 1)):
        r = orc.simulate(spec, np.zeros(3), ut, np.array([[0.5, 0.25 + dy, 0.25]]))
        assert r["col"] == col, dy
        assert r["clearance"] < 1e-10

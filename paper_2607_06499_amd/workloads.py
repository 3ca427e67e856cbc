"""Seeded synthetic workloads for the CE-MPPI replan path.

This module draws planner parameter sets and scenes shaped like the paper's
experiments (Sec. III: a differential-drive robot among circular obstacles,
static or moving, and a six-joint arm among moving spheres).  The paper's own
scenes exist only as figures and its arm runs on hardware, so every input
here is synthetic.  The module holds no arithmetic of the method itself: it
draws random numbers, places objects and moves obstacles (the world), and it
is the only code the GPU path and the CPU oracle share.

Every float handed to a planner is rounded to single precision here, so the
GPU (which computes in FP32) and the oracle (which promotes to FP64) start
from identical values.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

UNICYCLE, ARM6 = 0, 1
STATIC, DYNAMIC = 0, 1
FLAG_POSE_COST, FLAG_OBS_CONST_VEL = 1, 2
REF_TERMINAL, REF_FIRST_CONTACT = 0, 1
INF = float("inf")


def f32(x) -> float:
    return float(np.float32(x))


def f32a(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float32)


def dims(dynamics: int):
    """(n, m, p): state, control and task-space dimensions."""
    return (3, 2, 2) if dynamics == UNICYCLE else (12, 6, 3)


@dataclass
class PlannerSpec:
    """Planner parameters (Alg. 1 'Require' line) in single precision."""

    dynamics: int = UNICYCLE
    horizon: int = 30
    num_samples: int = 1024
    dt: float = 0.1
    lam: float = 1.0
    noise_chol: List[float] = field(default_factory=lambda: [0.0] * 36)
    u_min: List[float] = field(default_factory=lambda: [-INF] * 6)
    u_max: List[float] = field(default_factory=lambda: [INF] * 6)
    dbscan_eps: float = 0.3
    dbscan_min_pts: int = 10
    norm_eps: float = 1e-6
    scene_mode: int = STATIC
    history_len: int = 5
    v_obs_min: float = 1e-3
    ref_mode: int = REF_TERMINAL
    robot_radius: float = 0.0
    goal: List[float] = field(default_factory=lambda: [0.0] * 6)
    Q: List[float] = field(default_factory=lambda: [0.0] * 6)
    R: List[float] = field(default_factory=lambda: [0.0] * 6)
    Qf: List[float] = field(default_factory=lambda: [0.0] * 6)
    dh: List[float] = field(default_factory=lambda: [0.0] * 24)
    n_link_spheres: int = 8
    link_sphere_radius: float = 0.05
    q_limit: List[float] = field(default_factory=lambda: [math.pi] * 6)
    w_limit: float = 100.0
    max_obstacles: int = 64
    seed: int = 1
    stream_id: int = 0
    flags: int = 0

    @property
    def n(self) -> int:
        return dims(self.dynamics)[0]

    @property
    def m(self) -> int:
        return dims(self.dynamics)[1]

    @property
    def p(self) -> int:
        return dims(self.dynamics)[2]

    def rounded(self) -> "PlannerSpec":
        """Copy with every real parameter rounded to single precision."""
        s = dataclasses.replace(self)
        for f in dataclasses.fields(s):
            v = getattr(s, f.name)
            if isinstance(v, float):
                setattr(s, f.name, f32(v))
            elif isinstance(v, (list, tuple)) and v and isinstance(v[0], float):
                setattr(s, f.name, [f32(x) for x in v])
        return s

    def replace(self, **kw) -> "PlannerSpec":
        return dataclasses.replace(self, **kw).rounded()


def diag_chol(sigmas, m: int) -> List[float]:
    L = [0.0] * 36
    for i, s in enumerate(sigmas[:m]):
        L[i * m + i] = float(s)
    return L


# Table I bounds of the 2-D experiments: |v| <= 0.8 m/s, |omega| <= 7 rad/s.
TABLE1_UMIN = [-0.8, -7.0, -INF, -INF, -INF, -INF]
TABLE1_UMAX = [0.8, 7.0, INF, INF, INF, INF]


class ObstacleField:
    """Obstacles (centres, radii, velocities) in an axis-aligned box.  Moving
    obstacles keep a constant velocity and are mirrored at the walls."""

    def __init__(self, centres, radii, velocities, lo, hi):
        self.c = np.asarray(centres, dtype=np.float64).copy()
        self.r = np.asarray(radii, dtype=np.float64).copy()
        self.v = np.asarray(velocities, dtype=np.float64).copy()
        self.lo = np.asarray(lo, dtype=np.float64)
        self.hi = np.asarray(hi, dtype=np.float64)

    @property
    def n(self) -> int:
        return self.c.shape[0]

    def observation(self) -> np.ndarray:
        """Planner input rows (centre..., radius) in single precision."""
        return f32a(np.concatenate([self.c, self.r[:, None]], axis=1))

    def positions(self) -> np.ndarray:
        return f32a(self.c)

    def step(self, dt: float) -> None:
        self.c = self.c + self.v * dt
        for _ in range(2):
            low = self.c < self.lo
            self.c = np.where(low, 2 * self.lo - self.c, self.c)
            self.v = np.where(low, -self.v, self.v)
            high = self.c > self.hi
            self.c = np.where(high, 2 * self.hi - self.c, self.c)
            self.v = np.where(high, -self.v, self.v)

    def copy(self) -> "ObstacleField":
        return ObstacleField(self.c, self.r, self.v, self.lo, self.hi)


@dataclass
class Scene:
    spec: PlannerSpec
    x0: np.ndarray                 # initial state, float32
    U0: np.ndarray                 # initial nominal sequence [N][m], float32
    field: ObstacleField
    name: str = ""

    @property
    def obstacles(self) -> np.ndarray:
        return self.field.observation()


def _place_circles(rng, n, lo, hi, rmin, rmax, avoid, margin, speed=None):
    centres, radii, vels = [], [], []
    while len(centres) < n:
        r = rng.uniform(rmin, rmax)
        c = rng.uniform(lo, hi)
        if any(np.linalg.norm(c - np.asarray(a)) < r + margin for a in avoid):
            continue
        centres.append(c)
        radii.append(r)
        if speed is None:
            vels.append(np.zeros_like(c, dtype=float))
        else:
            s = rng.uniform(*speed)
            if len(lo) == 2:
                h = rng.uniform(0.0, 2 * math.pi)
                vels.append(np.array([s * math.cos(h), s * math.sin(h)]))
            else:
                d = rng.normal(size=3)
                vels.append(s * d / np.linalg.norm(d))
    dim = len(lo)
    return (np.array(centres, dtype=float).reshape(-1, dim), np.array(radii, dtype=float),
            np.array(vels, dtype=float).reshape(-1, dim))


def _unicycle_spec(**kw) -> PlannerSpec:
    base = dict(
        dynamics=UNICYCLE,
        noise_chol=diag_chol([0.5, 0.8], 2),
        u_min=list(TABLE1_UMIN),
        u_max=list(TABLE1_UMAX),
        Q=[1.0, 1.0, 0.0, 0.0, 0.0, 0.0],
        R=[0.01, 0.01, 0.0, 0.0, 0.0, 0.0],
        Qf=[1.0, 1.0, 0.0, 0.0, 0.0, 0.0],
    )
    base.update(kw)
    return PlannerSpec(**base).rounded()


def unicycle_static(seed: int = 1, num_samples: int = 1024) -> Scene:
    """Static 2-D scene: 10x10 m box, 8 circles r~U[0.3,0.8], start (0.5,0.5),
    goal (9.5,9.5); N=30, dt=0.1, lambda=1, eps=0.3, minPts=10, static rule."""
    rng = np.random.default_rng(seed)
    start, goal = np.array([0.5, 0.5]), np.array([9.5, 9.5])
    c, r, v = _place_circles(rng, 8, [0, 0], [10, 10], 0.3, 0.8, [start, goal], 0.5)
    spec = _unicycle_spec(horizon=30, num_samples=num_samples, dt=0.1, lam=1.0, dbscan_eps=0.3,
                          dbscan_min_pts=10, scene_mode=STATIC, goal=[9.5, 9.5, 0, 0, 0, 0],
                          seed=seed, stream_id=0)
    x0 = f32a([0.5, 0.5, math.pi / 4])
    return Scene(spec, x0, np.zeros((30, 2), np.float32), ObstacleField(c, r, v, [0, 0], [10, 10]),
                 "unicycle_static")


def unicycle_static_ahead(seed: int = 1, num_samples: int = 1024) -> Scene:
    """unicycle_static scene with obstacle 0 moved onto the start-goal segment 1.2 m
    ahead and a constant nominal (0.5, 0): the obstacle-directly-ahead case
    that makes Alg. 1 take the clustering branch."""
    s = unicycle_static(seed, num_samples)
    d = np.array([1.0, 1.0]) / math.sqrt(2.0)
    s.field.c[0] = np.array([0.5, 0.5]) + 1.2 * d
    U0 = np.zeros((s.spec.horizon, 2), np.float32)
    U0[:, 0] = 0.5
    return Scene(s.spec, s.x0, U0, s.field, "unicycle_static_ahead")


def unicycle_dynamic(seed: int = 1, num_samples: int = 8192) -> Scene:
    """Dynamic 2-D scene: 20x20 m box, 24 circles r~U[0.2,0.6] moving at
    U[0.2,1.0] m/s with wall reflection; N=50, dt=0.05, lambda=1, H=5,
    eps=0.25, minPts=20, dynamic rule; start (1,1), goal (19,19)."""
    rng = np.random.default_rng(seed)
    start, goal = np.array([1.0, 1.0]), np.array([19.0, 19.0])
    c, r, v = _place_circles(rng, 24, [0, 0], [20, 20], 0.2, 0.6, [start, goal], 1.0,
                             speed=(0.2, 1.0))
    spec = _unicycle_spec(horizon=50, num_samples=num_samples, dt=0.05, lam=1.0, dbscan_eps=0.25,
                          dbscan_min_pts=20, scene_mode=DYNAMIC, history_len=5,
                          goal=[19.0, 19.0, 0, 0, 0, 0], seed=seed, stream_id=0)
    x0 = f32a([1.0, 1.0, math.pi / 4])
    return Scene(spec, x0, np.zeros((50, 2), np.float32),
                 ObstacleField(c, r, v, [0, 0], [20, 20]), "unicycle_dynamic")


def unicycle_dynamic_ahead(seed: int = 1, num_samples: int = 8192) -> Scene:
    """unicycle_dynamic scene with obstacle 0 placed 1.0 m ahead of the start, moving
    along the robot's heading, and a constant nominal (0.6, 0): every replan
    of the probe takes the clustering branch with the dynamic rule."""
    s = unicycle_dynamic(seed, num_samples)
    d = np.array([1.0, 1.0]) / math.sqrt(2.0)
    s.field.c[0] = np.array([1.0, 1.0]) + 1.0 * d
    s.field.r[0] = 0.45
    s.field.v[0] = 0.4 * d
    U0 = np.zeros((s.spec.horizon, 2), np.float32)
    U0[:, 0] = 0.6
    return Scene(s.spec, s.x0, U0, s.field, "unicycle_dynamic_ahead")


# Six-joint arm with the joint-axis pattern of a UR-type manipulator:
# alpha = (pi/2, 0, 0, pi/2, -pi/2, 0), a = (0, -a2, -a3, 0, 0, 0),
# d = (d1, 0, 0, d4, d5, d6).
def arm_dh(lengths) -> List[float]:
    d1, a2, a3, d4, d5, d6 = [float(x) for x in lengths]
    rows = [
        (0.0, d1, math.pi / 2, 0.0),
        (-a2, 0.0, 0.0, 0.0),
        (-a3, 0.0, 0.0, 0.0),
        (0.0, d4, math.pi / 2, 0.0),
        (0.0, d5, -math.pi / 2, 0.0),
        (0.0, d6, 0.0, 0.0),
    ]
    return [v for row in rows for v in row]


def arm6_dynamic(seed: int = 1, num_samples: int = 4096) -> Scene:
    """Arm scene: seeded DH lengths U[0.08,0.45] m, joint-velocity noise
    sigma=0.3 rad/s, N=32, dt=0.05, 8 link spheres (r=0.05), 16 moving spheres
    r~U[0.04,0.12] at U[0.05,0.3] m/s in the cube [-0.6,0.6]^2 x [0,1.2],
    eps=0.35, minPts=16, dynamic rule; end-effector target in the cube."""
    rng = np.random.default_rng(seed)
    lengths = rng.uniform(0.08, 0.45, size=6)
    reach = float(np.sum(lengths[1:]))
    shoulder = np.array([0.0, 0.0, lengths[0]])
    lo, hi = np.array([-0.6, -0.6, 0.0]), np.array([0.6, 0.6, 1.2])
    while True:
        d = rng.normal(size=3)
        d[2] = abs(d[2])
        d /= np.linalg.norm(d)
        goal = shoulder + rng.uniform(0.3, 0.8) * reach * d
        if np.all(goal > lo) and np.all(goal < hi):
            break
    c, r, v = _place_circles(rng, 16, lo, hi, 0.04, 0.12, [np.zeros(3), shoulder, goal], 0.2,
                             speed=(0.05, 0.3))
    spec = PlannerSpec(
        dynamics=ARM6, horizon=32, num_samples=num_samples, dt=0.05, lam=1.0,
        noise_chol=diag_chol([0.3] * 6, 6), dbscan_eps=0.35, dbscan_min_pts=16,
        scene_mode=DYNAMIC, history_len=5, goal=list(goal) + [0.0] * 3,
        Q=[1.0] + [0.0] * 5, R=[0.0] * 6, Qf=[1.0] + [0.0] * 5, dh=arm_dh(lengths),
        n_link_spheres=8, link_sphere_radius=0.05, q_limit=[math.pi] * 6, w_limit=100.0,
        seed=seed, stream_id=0,
    ).rounded()
    x0 = np.zeros(12, np.float32)
    return Scene(spec, x0, np.zeros((32, 6), np.float32), ObstacleField(c, r, v, lo, hi), "arm6_dynamic")


def unicycle_crossing(seed: int = 1, side: int = 1, num_samples: int = 2048, distance: float = 1.5,
                      speed: float = 0.5) -> Scene:
    """unicycle_static robot with a single obstacle (r = 0.3) `distance` m
    straight ahead, crossing the path at `speed` m/s towards the robot's left
    (side +1) or right (side -1); constant nominal (0.7, 0), dynamic rule with
    H = 3.  The feasible rollouts pass on both sides, so DBSCAN finds two
    clusters at some steps and Eq. (18) chooses between them."""
    s = unicycle_static_ahead(seed, num_samples)
    h = math.pi / 4
    left = np.array([-math.sin(h), math.cos(h)])
    s.field.c = (np.asarray(s.x0[:2], np.float64) + distance * np.array([math.cos(h), math.sin(h)]))[None]
    s.field.r = np.array([0.3])
    s.field.v = (side * speed * left)[None]
    U0 = np.zeros_like(s.U0)
    U0[:, 0] = 0.7
    spec = s.spec.replace(scene_mode=DYNAMIC, history_len=3)
    return Scene(spec, s.x0, U0, s.field, "unicycle_crossing")


def arm6_dynamic_ahead(anchor, seed: int = 1, num_samples: int = 4096, gap: float = 0.03) -> Scene:
    """arm6_dynamic with obstacle 0 (r = 0.08) placed `gap` m from a link
    sphere of centre `anchor` (the caller's choice, e.g. the end-effector
    sphere at the start pose) and moving into the arm at 0.1 m/s: a share of
    the rollouts touch it, so Alg. 1 takes the clustering branch."""
    s = arm6_dynamic(seed, num_samples)
    n = np.array([1.0, 0.3, 0.2])
    n /= np.linalg.norm(n)
    r0 = 0.08
    s.field.c[0] = np.asarray(anchor, np.float64) + (s.spec.link_sphere_radius + r0 + gap) * n
    s.field.r[0] = r0
    s.field.v[0] = -0.1 * n
    return Scene(s.spec, s.x0, s.U0, s.field, "arm6_dynamic_ahead")


# ---------------------------------------------------------------- paper presets
def paper_unicycle_preset(scenario: int = 1, seed: int = 1) -> Scene:
    """Unicycle planner with the simulation parameters of Sec. III-A: K=300,
    N=30, dt=0.03, the Table I bounds, lambda 0.7 (scenario 1) or 0.01
    (scenario 2), stage weight Q=diag(10,10,0) and terminal weight
    diag(50,50,50) with no control term.  The layouts are synthetic:
    scenario 1 has one static obstacle on the start-goal line; scenario 2 a
    0.43 m/s obstacle moving along +x plus two static ones."""
    if scenario == 1:
        c = np.array([[0.55, 0.0]])
        r = np.array([0.2])
        v = np.zeros((1, 2))
        goal = [2.0, 0.0]
        lam, mode = 0.7, STATIC
    else:
        c = np.array([[0.45, 0.25], [2.0, 1.3], [3.0, 0.4]])
        r = np.array([0.2, 0.3, 0.3])
        v = np.array([[0.43, 0.0], [0.0, 0.0], [0.0, 0.0]])
        goal = [4.0, 2.0]
        lam, mode = 0.01, DYNAMIC
    spec = _unicycle_spec(horizon=30, num_samples=300, dt=0.03, lam=lam, dbscan_eps=0.3,
                          dbscan_min_pts=10, scene_mode=mode, history_len=5,
                          Q=[10.0, 10.0, 0.0, 0.0, 0.0, 0.0], R=[0.0] * 6,
                          Qf=[50.0, 50.0, 50.0, 0.0, 0.0, 0.0], goal=goal + [0.0] * 4,
                          seed=seed, stream_id=scenario)
    U0 = np.zeros((30, 2), np.float32)
    U0[:, 0] = 0.5
    return Scene(spec, f32a([0.0, 0.0, 0.0]), U0,
                 ObstacleField(c, r, v, [-1.0, -2.0], [5.0, 3.0]), f"paper_unicycle_{scenario}")


# published UR5e kinematic lengths (d1, a2, a3, d4, d5, d6) in metres
UR5E_LENGTHS = [0.1625, 0.425, 0.3922, 0.1333, 0.0997, 0.0996]


def paper_arm_preset(seed: int = 1) -> Scene:
    """Six-joint arm planner with the real-world parameters of Sec. III-C:
    K=50, N=12, dt=0.1, joint velocity bound 0.1 rad/s, joint position bound
    2 pi, lambda=0.05, DBSCAN eps=0.3 m on the end-effector feature, and the
    pose cost with (w_p, w_R, w_c) = (10, 3, 1000).  UR5e kinematic lengths;
    a synthetic target: a position with an obstacle sphere between it and the
    start pose (one more sphere elsewhere), and a tool-down orientation
    (half turn about a horizontal axis) turned 0.3 rad in yaw from the start."""
    rng = np.random.default_rng(70_000 + seed)
    bound = 0.1
    yaw = math.pi / 4 + 0.15
    spec = PlannerSpec(
        dynamics=ARM6, horizon=12, num_samples=50, dt=0.1, lam=0.05,
        noise_chol=diag_chol([0.05] * 6, 6), u_min=[-bound] * 6, u_max=[bound] * 6,
        dbscan_eps=0.3, dbscan_min_pts=5, scene_mode=STATIC, history_len=5,
        goal=[-0.6, -0.45, 0.4, math.pi * math.cos(yaw), math.pi * math.sin(yaw), 0.0],
        Q=[10.0, 3.0, 1000.0, 0.0, 0.0, 0.0], R=[0.0] * 6, Qf=[10.0, 3.0, 1000.0, 0.0, 0.0, 0.0],
        dh=arm_dh(UR5E_LENGTHS), n_link_spheres=8, link_sphere_radius=0.05,
        q_limit=[2.0 * math.pi] * 6, w_limit=100.0, seed=seed, stream_id=7, flags=FLAG_POSE_COST,
    ).rounded()
    q0 = np.array([0.0, -1.2, 1.4, -1.8, -1.57, 0.0]) + rng.normal(0.0, 0.02, 6)
    x0 = np.concatenate([q0, np.zeros(6)]).astype(np.float32)
    c = np.array([[-0.64, -0.22, 0.40], [-0.3, 0.2, 0.3]])
    r = np.array([0.05, 0.05])
    fld = ObstacleField(c, r, np.zeros((2, 3)), [-0.8, -0.8, 0.0], [0.8, 0.8, 1.2])
    return Scene(spec, x0, np.zeros((12, 6), np.float32), fld, "paper_arm")


def arm6_pose(seed: int = 1, num_samples: int = 4096) -> Scene:
    """arm6_dynamic with the pose cost of Sec. III-C (weights 10, 3, 1000;
    goal orientation a seeded rotation vector) and constant-velocity
    prediction of the moving spheres inside the rollouts."""
    s = arm6_dynamic(seed, num_samples)
    rng = np.random.default_rng(90_000 + seed)
    rv = rng.normal(size=3)
    rv *= rng.uniform(0.5, 2.5) / np.linalg.norm(rv)
    spec = s.spec.replace(goal=list(s.spec.goal[:3]) + list(rv), Q=[10.0, 3.0, 1000.0, 0.0, 0.0, 0.0],
                          Qf=[10.0, 3.0, 1000.0, 0.0, 0.0, 0.0],
                          flags=FLAG_POSE_COST | FLAG_OBS_CONST_VEL)
    return Scene(spec, s.x0, s.U0, s.field, "arm6_pose")


def unicycle_dynamic_cv(seed: int = 1, num_samples: int = 8192) -> Scene:
    """unicycle_dynamic with every obstacle predicted at constant velocity
    inside the rollouts (velocities from the observation history)."""
    s = unicycle_dynamic(seed, num_samples)
    return Scene(s.spec.replace(flags=FLAG_OBS_CONST_VEL), s.x0, s.U0, s.field, "unicycle_dynamic_cv")


def random_scene(seed: int, dynamics: int = UNICYCLE, num_samples: int = 512, horizon: int = 24,
                 n_obs: int = 6, scene_mode: int = STATIC, ref_mode: int = REF_TERMINAL,
                 clamp: bool = True, eps: Optional[float] = None, min_pts: Optional[int] = None,
                 lam: float = 1.0) -> Scene:
    """Small randomised problem for parity tests: the nominal sequence heads
    at an obstacle so that some rollouts collide and some pass on each side."""
    rng = np.random.default_rng(10_000 + seed)
    if dynamics == UNICYCLE:
        heading = rng.uniform(-math.pi, math.pi)
        x0 = np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), heading])
        d = np.array([math.cos(heading), math.sin(heading)])
        v_nom = rng.uniform(0.4, 0.7)
        dt = f32(rng.uniform(0.04, 0.1))
        ahead = x0[:2] + d * rng.uniform(0.4, 0.8) * v_nom * horizon * dt
        c, r, v = _place_circles(rng, max(n_obs - 1, 0), x0[:2] - 4, x0[:2] + 4, 0.2, 0.6,
                                 [x0[:2]], 0.4, speed=(0.1, 0.8))
        c0 = np.concatenate([[ahead], c]) if n_obs else np.zeros((0, 2))
        r0 = np.concatenate([[rng.uniform(0.2, 0.4)], r]) if n_obs else np.zeros(0)
        v0 = np.concatenate([[0.5 * d], v]) if n_obs else np.zeros((0, 2))
        spec = _unicycle_spec(
            horizon=horizon, num_samples=num_samples, dt=dt, lam=lam,
            dbscan_eps=eps if eps is not None else 0.3,
            dbscan_min_pts=min_pts if min_pts is not None else 8,
            scene_mode=scene_mode, ref_mode=ref_mode, history_len=4,
            goal=list(x0[:2] + d * 5.0) + [0.0] * 4, seed=seed, stream_id=seed % 7,
        )
        if not clamp:
            spec = spec.replace(u_min=[-INF] * 6, u_max=[INF] * 6)
        U0 = np.zeros((horizon, 2), np.float32)
        U0[:, 0] = v_nom
        U0[:, 1] = rng.normal(0, 0.2, size=horizon)
        fld = ObstacleField(c0, r0, v0, x0[:2] - 6, x0[:2] + 6)
        return Scene(spec, f32a(x0), f32a(U0), fld, "random_unicycle")
    lengths = rng.uniform(0.12, 0.4, size=6)
    dh = arm_dh(lengths)
    q0 = rng.uniform(-0.5, 0.5, size=6)
    spec = PlannerSpec(
        dynamics=ARM6, horizon=horizon, num_samples=num_samples, dt=f32(rng.uniform(0.03, 0.08)),
        lam=lam, noise_chol=diag_chol([0.3] * 6, 6), dbscan_eps=eps if eps is not None else 0.35,
        dbscan_min_pts=min_pts if min_pts is not None else 8, scene_mode=scene_mode,
        ref_mode=ref_mode, history_len=4, goal=list(rng.uniform(-0.4, 0.4, 3)) + [0.0] * 3,
        Q=[1.0] + [0.0] * 5, R=[0.01] * 6, Qf=[2.0] + [0.0] * 5, dh=dh, n_link_spheres=8,
        link_sphere_radius=0.05, q_limit=[1.5] * 6, w_limit=100.0, seed=seed,
        stream_id=seed % 5,
    )
    if clamp:
        spec = dataclasses.replace(spec, u_min=[-0.6] * 6, u_max=[0.6] * 6)
    spec = spec.rounded()
    # obstacles scattered around the reachable shell of the arm
    reach = float(np.sum(lengths[1:]))
    lo, hi = np.array([-1.0, -1.0, -0.2]), np.array([1.0, 1.0, 1.4])
    c, r, v = _place_circles(rng, n_obs, lo * reach, hi * reach, 0.05, 0.15, [], 0.0,
                             speed=(0.05, 0.3))
    U0 = f32a(rng.normal(0, 0.2, size=(horizon, 6)))
    x0 = np.concatenate([q0, np.zeros(6)])
    return Scene(spec, f32a(x0), U0, ObstacleField(c, r, v, lo * reach, hi * reach), "random_arm")


# ---------------------------------------------------------------- batched form
@dataclass
class BatchMember:
    scene: Scene
    kind: str


def batch_uneven(seed: int = 1, n_planners: int = 256) -> List[BatchMember]:
    """256 independent 2-D planners: K log-uniform in [256,16384], N uniform
    in [20,60], obstacle count uniform in [4,64]; even members static
    (unicycle_static style), odd members dynamic (unicycle_dynamic style)."""
    rng = np.random.default_rng(40_000 + seed)
    out = []
    for i in range(n_planners):
        K = int(round(math.exp(rng.uniform(math.log(256), math.log(16384)))))
        N = int(rng.integers(20, 61))
        n_obs = int(rng.integers(4, 65))
        sub = int(rng.integers(1, 2**31 - 1))
        srng = np.random.default_rng(sub)
        if i % 2 == 0:
            start, goal = np.array([0.5, 0.5]), np.array([9.5, 9.5])
            c, r, v = _place_circles(srng, n_obs, [0, 0], [10, 10], 0.3, 0.8, [start, goal], 0.5)
            spec = _unicycle_spec(horizon=N, num_samples=K, dt=0.1, lam=1.0, dbscan_eps=0.3,
                                  dbscan_min_pts=10, scene_mode=STATIC,
                                  goal=[9.5, 9.5, 0, 0, 0, 0], seed=sub, stream_id=i)
            x0 = f32a([0.5, 0.5, math.pi / 4])
            fld = ObstacleField(c, r, v, [0, 0], [10, 10])
        else:
            start, goal = np.array([1.0, 1.0]), np.array([19.0, 19.0])
            c, r, v = _place_circles(srng, n_obs, [0, 0], [20, 20], 0.2, 0.6, [start, goal], 1.0,
                                     speed=(0.2, 1.0))
            spec = _unicycle_spec(horizon=N, num_samples=K, dt=0.05, lam=1.0, dbscan_eps=0.25,
                                  dbscan_min_pts=20, scene_mode=DYNAMIC, history_len=5,
                                  goal=[19.0, 19.0, 0, 0, 0, 0], seed=sub, stream_id=i)
            x0 = f32a([1.0, 1.0, math.pi / 4])
            fld = ObstacleField(c, r, v, [0, 0], [20, 20])
        # an obstacle directly ahead, so most planners take the clustering branch
        ahead = x0[:2] + np.array([1.0, 1.0]) / math.sqrt(2.0) * srng.uniform(0.8, 1.4)
        fld.c[0] = ahead
        U0 = np.zeros((N, 2), np.float32)
        U0[:, 0] = 0.5
        out.append(BatchMember(Scene(spec, x0, U0, fld, f"batch_uneven[{i}]"),
                               "static" if i % 2 == 0 else "dynamic"))
    return out


# ---------------------------------------------------------------- served form
@dataclass
class SessionSpec:
    scene: Scene
    kind: str


def served_sessions(seed: int = 1, n_sessions: int = 512) -> List[SessionSpec]:
    """512 persistent sessions: 70 % 2-D planners (unicycle_static_ahead scene, K
    log-uniform in [1024,8192]) and 30 % arm planners (arm6_dynamic scene, K
    log-uniform in [1024,4096])."""
    rng = np.random.default_rng(50_000 + seed)
    out = []
    for i in range(n_sessions):
        sub = int(rng.integers(1, 2**31 - 1))
        if rng.uniform() < 0.7:
            K = int(round(math.exp(rng.uniform(math.log(1024), math.log(8192)))))
            s = unicycle_static_ahead(sub, K)
            s.spec = s.spec.replace(stream_id=i)
            out.append(SessionSpec(s, "unicycle"))
        else:
            K = int(round(math.exp(rng.uniform(math.log(1024), math.log(4096)))))
            s = arm6_dynamic(sub, K)
            s.spec = s.spec.replace(stream_id=i)
            out.append(SessionSpec(s, "arm"))
    return out


def poisson_arrivals(rate_hz: float, n: int, n_sessions: int, seed: int = 1):
    """Arrival times (s) and session ids of n Poisson-arrival requests."""
    rng = np.random.default_rng(60_000 + seed)
    t = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
    sess = rng.integers(0, n_sessions, size=n)
    return t, sess

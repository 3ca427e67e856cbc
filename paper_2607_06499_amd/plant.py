"""The simulated world a planner drives in a closed loop (host, FP64): the
robot plant that executes the applied control, and the obstacles moving in
their box.  The planner's own model uses the same kinematics (Sec. III-A for
the differential-drive robot, Sec. III-C for the joint-velocity arm); here
they advance the true state between replans."""
from __future__ import annotations

import math

import numpy as np


def unicycle_step(x, u, dt: float) -> np.ndarray:
    """Explicit-Euler differential drive: heading taken at the step start."""
    x = np.asarray(x, np.float64)
    v, w = float(u[0]), float(u[1])
    return np.array([x[0] + v * math.cos(x[2]) * dt, x[1] + v * math.sin(x[2]) * dt, x[2] + w * dt])


def arm_step(x, u, dt: float) -> np.ndarray:
    """Joint-velocity command: q <- q + u dt, qdot <- u."""
    x = np.asarray(x, np.float64)
    u = np.asarray(u, np.float64)
    return np.concatenate([x[:6] + u * dt, u])


def step(dynamics: int, x, u, dt: float) -> np.ndarray:
    return unicycle_step(x, u, dt) if dynamics == 0 else arm_step(x, u, dt)

"""ctypes marshalling for the FP64 oracle (test infrastructure only).

The problem description is any object (or mapping) carrying the planner
parameters by name: dynamics, horizon, num_samples, dt, lam, noise_chol,
u_min, u_max, dbscan_eps, dbscan_min_pts, norm_eps, scene_mode,
history_len, v_obs_min, ref_mode, robot_radius, goal, Q, R, Qf, dh,
n_link_spheres, link_sphere_radius, q_limit, w_limit, seed, stream_id and
(optional, default 0) flags.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cemppi_oracle.c")
_LIB = os.path.join(_HERE, "libcemppi_oracle.so")

UNICYCLE, ARM6 = 0, 1
FLAG_POSE_COST, FLAG_OBS_CONST_VEL = 1, 2
ST_FALLBACK, ST_ALL_COLLIDE, ST_NO_CLUSTER, ST_DYN_STATIC, ST_NONFINITE = 1, 2, 4, 8, 16

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


class OrcProblem(C.Structure):
    _fields_ = [
        ("dynamics", C.c_int32),
        ("N", C.c_int32),
        ("K", C.c_int32),
        ("dt", C.c_double),
        ("lam", C.c_double),
        ("L", C.c_double * 36),
        ("u_min", C.c_double * 6),
        ("u_max", C.c_double * 6),
        ("dbscan_eps", C.c_double),
        ("dbscan_min_pts", C.c_int32),
        ("norm_eps", C.c_double),
        ("scene_mode", C.c_int32),
        ("history_len", C.c_int32),
        ("v_obs_min", C.c_double),
        ("ref_mode", C.c_int32),
        ("robot_radius", C.c_double),
        ("goal", C.c_double * 6),
        ("Q", C.c_double * 6),
        ("R", C.c_double * 6),
        ("Qf", C.c_double * 6),
        ("dh", (C.c_double * 4) * 6),
        ("n_link_spheres", C.c_int32),
        ("link_sphere_radius", C.c_double),
        ("q_limit", C.c_double * 6),
        ("w_limit", C.c_double),
        ("seed", C.c_uint64),
        ("stream_id", C.c_uint32),
        ("flags", C.c_uint32),
    ]


def _p(ctype):
    return C.POINTER(ctype)


class OrcOut(C.Structure):
    _fields_ = [
        ("S", _p(C.c_double)),
        ("col", _p(C.c_int32)),
        ("first_obs", _p(C.c_int32)),
        ("p_term", _p(C.c_double)),
        ("p_first", _p(C.c_double)),
        ("eps_eff", _p(C.c_double)),
        ("clearance", _p(C.c_double)),
        ("v_idx", _p(C.c_int32)),
        ("z", _p(C.c_double)),
        ("g", _p(C.c_double)),
        ("ncount", _p(C.c_int32)),
        ("core", _p(C.c_int32)),
        ("label", _p(C.c_int32)),
        ("c_cap", C.c_int32),
        ("c_mean_cost", _p(C.c_double)),
        ("c_dir", _p(C.c_double)),
        ("c_size", _p(C.c_int32)),
        ("closest_force", C.c_int32),
        ("weight", _p(C.c_double)),
        ("U_new", _p(C.c_double)),
        ("U_next", _p(C.c_double)),
        ("u_out", _p(C.c_double)),
        ("branch", C.c_int32),
        ("n_col", C.c_int32),
        ("n_feas", C.c_int32),
        ("n_ref", C.c_int32),
        ("n_clusters", C.c_int32),
        ("selected", C.c_int32),
        ("selected_size", C.c_int32),
        ("closest", C.c_int32),
        ("rule", C.c_int32),
        ("h_used", C.c_int32),
        ("status", C.c_uint32),
        ("margin", C.c_double),
        ("closest_margin", C.c_double),
        ("ref_point", C.c_double * 3),
        ("v_obs", C.c_double * 3),
        ("v_obs_hat", C.c_double * 3),
        ("s_min", C.c_double),
    ]


_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = [
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-Wall", "-o", _LIB, _SRC, "-lm",
        ]
        subprocess.run(cmd, check=True)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(_LIB)
    lib.orc_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.orc_uniform.argtypes = [C.c_uint32]
    lib.orc_uniform.restype = C.c_double
    lib.orc_box_muller.argtypes = [C.c_uint32, C.c_uint32, _p(C.c_double), _p(C.c_double)]
    lib.orc_noise_blocks.argtypes = [C.c_int32, C.c_int32]
    lib.orc_noise_blocks.restype = C.c_int32
    lib.orc_noise_words.argtypes = [_p(OrcProblem), C.c_uint32, C.c_int32, _u32p]
    lib.orc_rollout_noise.argtypes = [_p(OrcProblem), C.c_uint32, C.c_int32, _f64p, _f64p]
    lib.orc_unicycle_step.argtypes = [_f64p, _f64p, C.c_double, _f64p]
    lib.orc_arm_frames.argtypes = [_f64p, _f64p, _f64p, _f64p]
    lib.orc_arm_spheres.argtypes = [_f64p, C.c_int32, _f64p]
    lib.orc_simulate.argtypes = [
        _p(OrcProblem), _f64p, _f64p, _f64p, C.c_int32, C.c_void_p, _p(C.c_double),
        _p(C.c_int32), _p(C.c_int32), _f64p, _f64p, _p(C.c_double),
    ]
    lib.orc_simulate_moving.argtypes = [
        _p(OrcProblem), _f64p, _f64p, _f64p, C.c_void_p, C.c_int32, C.c_void_p, _p(C.c_double),
        _p(C.c_int32), _p(C.c_int32), _f64p, _f64p, _p(C.c_double),
    ]
    lib.orc_rotvec_quat.argtypes = [_f64p, _f64p]
    lib.orc_rot_quat.argtypes = [_f64p, _f64p]
    lib.orc_quat_angle.argtypes = [_f64p, _f64p]
    lib.orc_quat_angle.restype = C.c_double
    lib.orc_closest_obstacle.argtypes = [_p(OrcProblem), _f64p, _f64p, C.c_int32]
    lib.orc_closest_obstacle.restype = C.c_int32
    lib.orc_closest_obstacle_margin.argtypes = [_p(OrcProblem), _f64p, _f64p, C.c_int32,
                                                _p(C.c_double)]
    lib.orc_closest_obstacle_margin.restype = C.c_int32
    lib.orc_select_cluster.argtypes = [
        _p(OrcProblem), C.c_int32, _i32p, C.c_int32, _f64p, _f64p, _f64p, C.c_int32, C.c_int32,
        C.c_int32, _p(OrcOut),
    ]
    lib.orc_select_cluster.restype = C.c_int32
    lib.orc_obstacle_velocity.argtypes = [
        _f64p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double, _f64p,
    ]
    lib.orc_dbscan.argtypes = [_f64p, C.c_int32, C.c_int32, C.c_double, C.c_int32, _i32p, _i32p, _i32p]
    lib.orc_dbscan.restype = C.c_int32
    lib.orc_weighted_update.argtypes = [
        C.c_int32, _i32p, _f64p, _f64p, C.c_int32, C.c_int32, C.c_double, _f64p, _f64p, _f64p,
        _p(C.c_double),
    ]
    lib.orc_replan.argtypes = [
        _p(OrcProblem), _f64p, _f64p, _f64p, C.c_int32, _f64p, C.c_int32, C.c_uint32, _p(OrcOut),
    ]
    lib.orc_replan.restype = C.c_int32
    lib.orc_replan_from_rollouts.argtypes = [
        _p(OrcProblem), _f64p, _f64p, _f64p, C.c_int32, _f64p, C.c_int32, _f64p, _i32p, _i32p,
        _f64p, _f64p, _f64p, _p(OrcOut),
    ]
    lib.orc_replan_from_rollouts.restype = C.c_int32
    _lib = lib
    return lib


def _get(spec, name, default=None):
    if isinstance(spec, dict):
        return spec.get(name, default)
    return getattr(spec, name, default)


def dims(dynamics: int):
    return (3, 2, 2) if int(dynamics) == UNICYCLE else (12, 6, 3)


def make_problem(spec) -> OrcProblem:
    """Promote the (single-precision) planner parameters to double exactly."""
    P = OrcProblem()
    P.dynamics = int(_get(spec, "dynamics"))
    P.N = int(_get(spec, "horizon"))
    P.K = int(_get(spec, "num_samples"))
    P.dt = float(np.float32(_get(spec, "dt")))
    P.lam = float(np.float32(_get(spec, "lam")))
    L = np.asarray(_get(spec, "noise_chol"), dtype=np.float32).astype(np.float64).ravel()
    for i in range(36):
        P.L[i] = L[i] if i < L.size else 0.0
    for name in ("u_min", "u_max", "goal", "Q", "R", "Qf", "q_limit"):
        v = np.asarray(_get(spec, name), dtype=np.float32).astype(np.float64).ravel()
        arr = getattr(P, name)
        for i in range(6):
            arr[i] = v[i] if i < v.size else 0.0
    P.dbscan_eps = float(np.float32(_get(spec, "dbscan_eps")))
    P.dbscan_min_pts = int(_get(spec, "dbscan_min_pts"))
    P.norm_eps = float(np.float32(_get(spec, "norm_eps")))
    P.scene_mode = int(_get(spec, "scene_mode"))
    P.history_len = int(_get(spec, "history_len"))
    P.v_obs_min = float(np.float32(_get(spec, "v_obs_min")))
    P.ref_mode = int(_get(spec, "ref_mode"))
    P.robot_radius = float(np.float32(_get(spec, "robot_radius")))
    dh = np.asarray(_get(spec, "dh"), dtype=np.float32).astype(np.float64).reshape(6, 4)
    for i in range(6):
        for c in range(4):
            P.dh[i][c] = dh[i, c]
    P.n_link_spheres = int(_get(spec, "n_link_spheres"))
    P.link_sphere_radius = float(np.float32(_get(spec, "link_sphere_radius")))
    P.w_limit = float(np.float32(_get(spec, "w_limit")))
    P.seed = int(_get(spec, "seed")) & 0xFFFFFFFFFFFFFFFF
    P.stream_id = int(_get(spec, "stream_id")) & 0xFFFFFFFF
    P.flags = int(_get(spec, "flags", 0) or 0) & 0xFFFFFFFF
    return P


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr, key) -> np.ndarray:
    lib = load()
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(c, k, out)
    return out


def uniform(w: int) -> float:
    return load().orc_uniform(int(w) & 0xFFFFFFFF)


def box_muller(wa: int, wb: int):
    a, b = C.c_double(), C.c_double()
    load().orc_box_muller(int(wa) & 0xFFFFFFFF, int(wb) & 0xFFFFFFFF, C.byref(a), C.byref(b))
    return a.value, b.value


def noise_blocks(N: int, m: int) -> int:
    return load().orc_noise_blocks(int(N), int(m))


def noise_words(spec, step: int, k: int) -> np.ndarray:
    lib = load()
    P = make_problem(spec)
    _, m, _ = dims(P.dynamics)
    out = np.zeros(4 * noise_blocks(P.N, m), dtype=np.uint32)
    lib.orc_noise_words(C.byref(P), int(step) & 0xFFFFFFFF, int(k), out)
    return out


def rollout_noise(spec, step: int, k: int):
    """Return (gauss [N][m], eps [N][m]) of rollout k."""
    lib = load()
    P = make_problem(spec)
    _, m, _ = dims(P.dynamics)
    g = np.zeros(P.N * m)
    e = np.zeros(P.N * m)
    lib.orc_rollout_noise(C.byref(P), int(step) & 0xFFFFFFFF, int(k), g, e)
    return g.reshape(P.N, m), e.reshape(P.N, m)


def unicycle_step(x, u, dt):
    out = np.zeros(3)
    load().orc_unicycle_step(_f64(x), _f64(u), float(dt), out)
    return out


def arm_frames(q, dh):
    org = np.zeros((7, 3))
    rot = np.zeros((3, 3))
    load().orc_arm_frames(_f64(q), _f64(np.asarray(dh).reshape(6, 4)), org, rot)
    return org, rot


def arm_spheres(origins, ns: int):
    out = np.zeros((ns, 3))
    load().orc_arm_spheres(_f64(origins), int(ns), out)
    return out


def simulate(spec, x0, ut, obs, vel=None):
    """One rollout with the applied controls ut [N][m]; obstacles move with
    velocities vel [n_obs][p] (None: frozen).  Returns a dict."""
    lib = load()
    P = make_problem(spec)
    n, m, p = dims(P.dynamics)
    obs = _f64(obs).reshape(-1, p + 1) if np.size(obs) else np.zeros((0, p + 1))
    traj = np.zeros((P.N + 1, n))
    S, col, fo, clr = C.c_double(), C.c_int32(), C.c_int32(), C.c_double()
    pT, pF = np.zeros(p), np.zeros(p)
    v = None
    if vel is not None:
        v = np.ascontiguousarray(_f64(vel).reshape(obs.shape[0], p).ravel())
    lib.orc_simulate_moving(
        C.byref(P), _f64(x0), _f64(ut).ravel(), np.ascontiguousarray(obs.ravel()),
        v.ctypes.data_as(C.c_void_p) if v is not None and v.size else None, obs.shape[0],
        traj.ctypes.data_as(C.c_void_p), C.byref(S), C.byref(col), C.byref(fo), pT, pF, C.byref(clr),
    )
    return dict(traj=traj, S=S.value, col=col.value, first_obs=fo.value, p_term=pT, p_first=pF,
                clearance=clr.value)


def rotvec_quat(r) -> np.ndarray:
    q = np.zeros(4)
    load().orc_rotvec_quat(_f64(r), q)
    return q


def rot_quat(R) -> np.ndarray:
    q = np.zeros(4)
    load().orc_rot_quat(np.ascontiguousarray(_f64(R).reshape(3, 3)), q)
    return q


def quat_angle(a, b) -> float:
    return float(load().orc_quat_angle(_f64(a), _f64(b)))


def closest_obstacle(spec, x0, obs) -> int:
    P = make_problem(spec)
    _, _, p = dims(P.dynamics)
    obs = _f64(obs).reshape(-1, p + 1)
    return load().orc_closest_obstacle(C.byref(P), _f64(x0), np.ascontiguousarray(obs.ravel()),
                                       obs.shape[0])


def closest_obstacle_margin(spec, x0, obs):
    """(o*, second-smallest minus smallest surface clearance)."""
    P = make_problem(spec)
    _, _, p = dims(P.dynamics)
    obs = _f64(obs).reshape(-1, p + 1)
    mg = C.c_double()
    i = load().orc_closest_obstacle_margin(C.byref(P), _f64(x0),
                                           np.ascontiguousarray(obs.ravel()) if obs.size else np.zeros(1),
                                           obs.shape[0], C.byref(mg))
    return i, mg.value


def select_cluster(spec, labels, S_v, g, obs, hist=None, closest: int = 0, c_cap: int = 4096):
    """Cluster statistics and selection on given labels of the feasible set
    (S_v [V] costs, g [V][p] directions); obs/hist as in replan."""
    lib = load()
    P = make_problem(spec)
    _, _, p = dims(P.dynamics)
    lab = np.ascontiguousarray(np.asarray(labels, dtype=np.int32))
    V = len(lab)
    M = int(lab.max()) + 1 if V else 0
    if M == 0:
        raise ValueError("select_cluster needs at least one cluster")
    obs = _f64(obs).reshape(-1, p + 1) if np.size(obs) else np.zeros((0, p + 1))
    n_obs = obs.shape[0]
    if hist is None:
        hist = obs[None, :, :p]
    hist = _f64(hist).reshape(-1, n_obs, p) if n_obs else np.zeros((1, 0, p))
    r = dict(c_mean_cost=np.zeros(c_cap), c_dir=np.zeros((c_cap, p)), c_size=np.zeros(c_cap, np.int32))
    o = OrcOut()
    for name, arr in r.items():
        setattr(o, name, _ptr(arr, C.c_int32 if arr.dtype == np.int32 else C.c_double))
    o.c_cap = c_cap
    o.status = 0
    o.h_used = 0
    o.margin = np.inf
    sel = lib.orc_select_cluster(C.byref(P), V, lab, M, _f64(S_v), np.ascontiguousarray(_f64(g).ravel()),
                                 np.ascontiguousarray(hist.ravel()) if hist.size else np.zeros(1),
                                 hist.shape[0], n_obs, int(closest), C.byref(o))
    for name in ("c_mean_cost", "c_dir", "c_size"):
        r[name] = r[name][:min(M, c_cap)]
    r.update(selected=sel, selected_size=o.selected_size, rule=o.rule, h_used=o.h_used,
             status=o.status, margin=o.margin, n_clusters=M,
             v_obs=np.array(o.v_obs[:p]), v_obs_hat=np.array(o.v_obs_hat[:p]))
    return r


def obstacle_velocity(hist, idx: int, H: int, dt: float) -> np.ndarray:
    """hist [h_avail][n_obs][p], newest first."""
    hist = _f64(hist)
    h_avail, n_obs, p = hist.shape
    v = np.zeros(3)
    load().orc_obstacle_velocity(np.ascontiguousarray(hist.ravel()), h_avail, n_obs, p, int(idx),
                                 int(H), float(dt), v)
    return v[:p]


def dbscan(z, eps: float, min_pts: int):
    """Return (labels, core, ncount, M) for features z [V][p]."""
    z = _f64(z)
    V = z.shape[0]
    p = z.shape[1] if z.ndim == 2 else 1
    nc = np.zeros(max(V, 1), dtype=np.int32)
    co = np.zeros(max(V, 1), dtype=np.int32)
    lb = np.zeros(max(V, 1), dtype=np.int32)
    M = load().orc_dbscan(np.ascontiguousarray(z.ravel()) if V else np.zeros(1), V, p,
                          float(np.float32(eps)), int(min_pts), nc, co, lb)
    return lb[:V], co[:V].astype(bool), nc[:V], M


def weighted_update(set_idx, S, eps_eff, lam, U):
    """set_idx: rollout indices; S [K]; eps_eff [K][N][m]; U [N][m]."""
    E = _f64(eps_eff)
    K, N, m = E.shape
    idx = np.ascontiguousarray(np.asarray(set_idx, dtype=np.int32))
    Un = np.zeros(N * m)
    w = np.zeros(K)
    smin = C.c_double()
    load().orc_weighted_update(len(idx), idx if len(idx) else np.zeros(1, np.int32), _f64(S),
                               np.ascontiguousarray(E.ravel()), N, m, float(lam),
                               _f64(U).ravel(), Un, w, C.byref(smin))
    return Un.reshape(N, m), w, smin.value


# ---------------------------------------------------------------- full replan
def replan(spec, x_t, U, obs, hist=None, step: int = 0, c_cap: int = 4096, rollouts=None,
           closest=None):
    """Run Alg. 1 once.  obs [n_obs][p+1]; hist [h_avail][n_obs][p] newest
    first (defaults to the current positions alone).  With ``rollouts`` (a
    dict of S, col, first_obs, p_term, p_first, eps_eff) the rollout stage is
    skipped and those records are used.  ``closest`` (an obstacle index, or
    -1) replaces the computed o*, to resolve a near tie the way another
    implementation did.  Returns a dict."""
    lib = load()
    P = make_problem(spec)
    n, m, p = dims(P.dynamics)
    K, N = P.K, P.N
    obs = _f64(obs).reshape(-1, p + 1) if np.size(obs) else np.zeros((0, p + 1))
    n_obs = obs.shape[0]
    if hist is None:
        hist = obs[None, :, :p]
    hist = _f64(hist).reshape(-1, n_obs, p) if n_obs else np.zeros((1, 0, p))
    h_avail = hist.shape[0]
    r = dict(
        S=np.zeros(K), col=np.zeros(K, np.int32), first_obs=np.zeros(K, np.int32),
        p_term=np.zeros((K, p)), p_first=np.zeros((K, p)), eps_eff=np.zeros((K, N, m)),
        clearance=np.zeros(K), v_idx=np.zeros(K, np.int32), z=np.zeros((K, p)), g=np.zeros((K, p)),
        ncount=np.zeros(K, np.int32), core=np.zeros(K, np.int32), label=np.zeros(K, np.int32),
        c_mean_cost=np.zeros(c_cap), c_dir=np.zeros((c_cap, p)), c_size=np.zeros(c_cap, np.int32),
        weight=np.zeros(K), U_new=np.zeros((N, m)), U_next=np.zeros((N, m)), u_out=np.zeros(m),
    )
    o = OrcOut()
    for name, arr in r.items():
        ct = C.c_int32 if arr.dtype == np.int32 else C.c_double
        setattr(o, name, _ptr(arr, ct))
    o.c_cap = c_cap
    o.closest_force = -2 if closest is None else int(closest)
    obs_flat = np.ascontiguousarray(obs.ravel()) if n_obs else np.zeros(1)
    hist_flat = np.ascontiguousarray(hist.ravel()) if hist.size else np.zeros(1)
    if rollouts is None:
        rc = lib.orc_replan(C.byref(P), _f64(x_t), _f64(U).ravel(), obs_flat, n_obs, hist_flat,
                            h_avail, int(step) & 0xFFFFFFFF, C.byref(o))
    else:
        ro = rollouts
        rc = lib.orc_replan_from_rollouts(
            C.byref(P), _f64(x_t), _f64(U).ravel(), obs_flat, n_obs, hist_flat, h_avail,
            _f64(ro["S"]), np.ascontiguousarray(ro["col"], dtype=np.int32),
            np.ascontiguousarray(ro["first_obs"], dtype=np.int32), _f64(ro["p_term"]).ravel(),
            _f64(ro["p_first"]).ravel(), _f64(ro["eps_eff"]).ravel(), C.byref(o))
        for name in ("S", "col", "first_obs", "p_term", "p_first", "eps_eff"):
            r[name] = np.asarray(ro[name]).copy()
    if rc != 0:
        raise ValueError("oracle rejected the problem")
    nV = o.n_feas
    M = o.n_clusters
    for name in ("v_idx", "z", "g", "ncount", "core", "label"):
        r[name] = r[name][:nV]
    r["core"] = r["core"].astype(bool)
    for name in ("c_mean_cost", "c_dir", "c_size"):
        r[name] = r[name][:min(M, c_cap)]
    for name in ("branch", "n_col", "n_feas", "n_ref", "n_clusters", "selected", "selected_size",
                 "closest", "rule", "h_used", "status", "margin", "closest_margin", "s_min"):
        r[name] = getattr(o, name)
    r["ref_point"] = np.array(o.ref_point[:p])
    r["v_obs"] = np.array(o.v_obs[:p])
    r["v_obs_hat"] = np.array(o.v_obs_hat[:p])
    return r

"""ctypes binding of libcemppi.so: the C-ABI entry points under their own
names, plus a small ``Planner`` wrapper that marshals torch tensors (device
memory) and the current torch stream.  Argument marshalling only: every step
of the replan runs in the HIP library, and nothing here falls back to any
other implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcemppi.so")

ABI_VERSION = 1
NOALLOC_MAX_POINTS = 16384
CE_OK, CE_EINVAL, CE_ENOMEM, CE_EDEVICE, CE_EUNSUPPORTED, CE_EBUSY = range(6)
DYN_UNICYCLE, DYN_ARM6 = 0, 1
SCENE_STATIC, SCENE_DYNAMIC = 0, 1
REF_TERMINAL, REF_FIRST_CONTACT = 0, 1
FLAG_POSE_COST, FLAG_OBS_CONST_VEL = 1, 2
BRANCH_CLUSTER, BRANCH_FALLBACK, BRANCH_ALL_COLLIDE = 0, 1, 2
STATUS_FALLBACK, STATUS_ALL_COLLIDE, STATUS_NO_CLUSTER, STATUS_DYN_STATIC, STATUS_NONFINITE = (
    1, 2, 4, 8, 16)
LAUNCH_GRAPH, LAUNCH_DIRECT = 0, 1
DBSCAN_AUTO, DBSCAN_WINDOW, DBSCAN_BITMAP, DBSCAN_TILED = 0, 1, 2, 3
SERVE_BATCHED, SERVE_PLAIN = 0, 1
(DBG_COST, DBG_COLLIDE, DBG_FIRST_OBS, DBG_P_TERM, DBG_P_FIRST, DBG_EPS, DBG_V_IDX, DBG_Z, DBG_G,
 DBG_NCOUNT, DBG_LABEL, DBG_CLUSTER_COST, DBG_CLUSTER_DIR, DBG_CLUSTER_SIZE, DBG_TREES) = range(15)


class CeMppiConfig(C.Structure):
    _fields_ = [
        ("abi_version", C.c_uint32),
        ("dynamics", C.c_int32),
        ("horizon", C.c_int32),
        ("num_samples", C.c_int32),
        ("dt", C.c_float),
        ("lam", C.c_float),
        ("noise_chol", C.c_float * 36),
        ("u_min", C.c_float * 6),
        ("u_max", C.c_float * 6),
        ("dbscan_eps", C.c_float),
        ("dbscan_min_pts", C.c_int32),
        ("norm_eps", C.c_float),
        ("scene_mode", C.c_int32),
        ("history_len", C.c_int32),
        ("v_obs_min", C.c_float),
        ("ref_mode", C.c_int32),
        ("max_obstacles", C.c_int32),
        ("robot_radius", C.c_float),
        ("goal", C.c_float * 6),
        ("Q", C.c_float * 6),
        ("R", C.c_float * 6),
        ("Qf", C.c_float * 6),
        ("dh", (C.c_float * 4) * 6),
        ("n_link_spheres", C.c_int32),
        ("link_sphere_radius", C.c_float),
        ("q_limit", C.c_float * 6),
        ("w_limit", C.c_float),
        ("seed", C.c_uint64),
        ("stream_id", C.c_uint32),
        ("device", C.c_int32),
        ("flags", C.c_uint32),
    ]


class CeMppiInfo(C.Structure):
    _fields_ = [
        ("branch", C.c_int32),
        ("n_collide", C.c_int32),
        ("n_feasible", C.c_int32),
        ("n_ref", C.c_int32),
        ("n_clusters", C.c_int32),
        ("selected", C.c_int32),
        ("selected_size", C.c_int32),
        ("closest", C.c_int32),
        ("rule", C.c_int32),
        ("history_used", C.c_int32),
        ("status", C.c_uint32),
        ("step", C.c_uint32),
        ("margin", C.c_float),
        ("s_min", C.c_float),
        ("ref_point", C.c_float * 3),
        ("v_obs", C.c_float * 3),
        ("v_obs_hat", C.c_float * 3),
        ("weight_sum", C.c_float),
    ]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_}
        for k in ("ref_point", "v_obs", "v_obs_hat"):
            d[k] = np.array(list(d[k]), dtype=np.float32)
        return d


class CeMppiBatchIO(C.Structure):
    _fields_ = [
        ("x_t", C.c_void_p),
        ("obstacles", C.c_void_p),
        ("n_obs", C.c_int32),
        ("reserved", C.c_int32),
        ("u_out", C.c_void_p),
        ("U_out", C.c_void_p),
        ("info", C.c_void_p),
    ]


class CeMppiBatchTuning(C.Structure):
    _fields_ = [
        ("colg", C.c_int32),
        ("tile_blocks_per_cu", C.c_int32),
        ("roll_blocks_per_cu", C.c_int32),
        ("roll_per_wave", C.c_int32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class CeMppiServerConfig(C.Structure):
    _fields_ = [
        ("device", C.c_int32),
        ("max_batch", C.c_int32),
        ("max_inflight", C.c_int32),
        ("mode", C.c_int32),
        ("memory_budget", C.c_uint64),
    ]


class CeMppiServerStats(C.Structure):
    _fields_ = [
        ("launches", C.c_uint64),
        ("served", C.c_uint64),
        ("mean_batch", C.c_double),
        ("max_batch", C.c_int32),
        ("max_inflight", C.c_int32),
        ("sessions", C.c_int32),
        ("reserved", C.c_int32),
        ("session_bytes", C.c_uint64),
        ("budget_bytes", C.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}


INFO_BYTES = C.sizeof(CeMppiInfo)
_vp = C.c_void_p

_lib = None


class CeMppiError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed: status {status} ({msg})")
        self.status = status


def load():
    """Open libcemppi.so (built in-tree by ``build.py``); raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is missing: build it with paper_2607_06499_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    sig = {
        "ce_mppi_config_init": [C.POINTER(CeMppiConfig), C.c_int32],
        "ce_mppi_create": [C.POINTER(CeMppiConfig), C.POINTER(_vp)],
        "ce_mppi_replan": [_vp, _vp, _vp, C.c_int32, _vp, _vp, _vp, _vp],
        "ce_mppi_set_nominal": [_vp, _vp, _vp],
        "ce_mppi_get_nominal": [_vp, _vp, _vp],
        "ce_mppi_reset_history": [_vp, _vp],
        "ce_mppi_set_history": [_vp, _vp, C.c_int32, C.c_int32, _vp],
        "ce_mppi_set_step": [_vp, C.c_uint64, _vp],
        "ce_mppi_state_size": [_vp, C.POINTER(C.c_size_t)],
        "ce_mppi_get_state": [_vp, _vp, C.c_size_t, _vp],
        "ce_mppi_set_state": [_vp, _vp, C.c_size_t, _vp],
        "ce_mppi_debug_get": [_vp, C.c_int32, _vp, C.c_size_t, _vp],
        "ce_mppi_stage_noise": [_vp, C.c_uint32, _vp, _vp, _vp],
        "ce_mppi_replan_from_rollouts": [_vp, _vp, _vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp,
                                         _vp, _vp, _vp, _vp],
        "ce_mppi_stage_dbscan": [_vp, _vp, C.c_int32, _vp, _vp, _vp, _vp],
        "ce_mppi_dbscan_noalloc": [C.c_int32, _vp, C.c_int32, C.c_int32, C.c_float, C.c_int32, _vp, _vp,
                                   _vp, _vp],
        "ce_mppi_set_launch_mode": [_vp, C.c_int32],
        "ce_mppi_set_dbscan_mode": [_vp, C.c_int32],
        "ce_mppi_get_dbscan_path": [_vp, C.POINTER(C.c_int32)],
        "ce_mppi_tune_launch": [_vp, _vp, _vp, C.c_int32, _vp, C.c_int32, _vp,
                                C.POINTER(C.c_double), C.POINTER(C.c_double)],
        "ce_mppi_timing_enable": [_vp, C.c_int32],
        "ce_mppi_timing_read": [_vp, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                C.POINTER(C.c_double), C.POINTER(C.c_int32)],
        "ce_mppi_time_rollout": [_vp, _vp, _vp, C.c_int32, C.c_int32, _vp, C.POINTER(C.c_double)],
        "ce_mppi_timing_read_each": [_vp, C.c_int32, _vp, _vp, _vp, C.POINTER(C.c_int32)],
        "ce_mppi_batch_create": [C.POINTER(_vp), C.c_int32, C.POINTER(_vp)],
        "ce_mppi_batch_replan": [_vp, C.POINTER(CeMppiBatchIO), _vp],
        "ce_mppi_batch_replan_subset": [_vp, C.POINTER(C.c_int32), C.c_int32, C.POINTER(CeMppiBatchIO),
                                        _vp],
        "ce_mppi_batch_set_tuning": [_vp, C.POINTER(CeMppiBatchTuning)],
        "ce_mppi_server_create": [C.POINTER(CeMppiServerConfig), C.POINTER(_vp)],
        "ce_mppi_server_open_session": [_vp, C.POINTER(CeMppiConfig), _vp, C.POINTER(C.c_int32)],
        "ce_mppi_server_start": [_vp],
        "ce_mppi_server_submit": [_vp, C.c_int32, _vp, _vp, C.c_int32, C.POINTER(C.c_uint64)],
        "ce_mppi_server_wait": [_vp, C.c_uint64, _vp, _vp, C.POINTER(C.c_double)],
        "ce_mppi_server_run_trace": [_vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
        "ce_mppi_server_get_stats": [_vp, C.POINTER(CeMppiServerStats)],
        "ce_mppi_batch_get_tuning": [_vp, C.POINTER(CeMppiBatchTuning)],
        "ce_mppi_batch_autotune": [_vp, C.POINTER(CeMppiBatchIO), C.c_int32, _vp,
                                   C.POINTER(CeMppiBatchTuning), C.POINTER(C.c_double)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int32
    lib.ce_mppi_destroy.argtypes = [_vp]
    lib.ce_mppi_destroy.restype = None
    lib.ce_mppi_batch_destroy.argtypes = [_vp]
    lib.ce_mppi_batch_destroy.restype = None
    lib.ce_mppi_server_destroy.argtypes = [_vp]
    lib.ce_mppi_server_destroy.restype = None
    lib.ce_mppi_server_session_planner.argtypes = [_vp, C.c_int32]
    lib.ce_mppi_server_session_planner.restype = _vp
    lib.ce_mppi_status_string.argtypes = [C.c_int32]
    lib.ce_mppi_status_string.restype = C.c_char_p
    lib.ce_mppi_last_error.argtypes = []
    lib.ce_mppi_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(fn: str, status: int):
    if status != CE_OK:
        msg = load().ce_mppi_last_error().decode()
        raise CeMppiError(fn, status, msg)


# ----------------------------------------------------------------- raw C-ABI
def ce_mppi_config_init(dynamics: int) -> CeMppiConfig:
    cfg = CeMppiConfig()
    _check("ce_mppi_config_init", load().ce_mppi_config_init(C.byref(cfg), int(dynamics)))
    return cfg


def ce_mppi_create(cfg: CeMppiConfig) -> int:
    h = _vp()
    _check("ce_mppi_create", load().ce_mppi_create(C.byref(cfg), C.byref(h)))
    return h.value


def ce_mppi_replan(planner: int, x_t: int, obstacles: int, n_obs: int, u_out: int, U_out: int,
                   info: int, stream: int) -> None:
    _check("ce_mppi_replan",
           load().ce_mppi_replan(planner, x_t, obstacles, n_obs, u_out, U_out, info, stream))


def ce_mppi_destroy(planner: int) -> None:
    load().ce_mppi_destroy(planner)


def ce_mppi_status_string(status: int) -> str:
    return load().ce_mppi_status_string(int(status)).decode()


def ce_mppi_last_error() -> str:
    return load().ce_mppi_last_error().decode()


# ----------------------------------------------------------------- marshalling
def config_from_spec(spec, device: int = 0) -> CeMppiConfig:
    """Fill a CeMppiConfig from a planner spec object (attributes named as in
    ``workloads.PlannerSpec``)."""
    cfg = ce_mppi_config_init(int(spec.dynamics))
    cfg.horizon = int(spec.horizon)
    cfg.num_samples = int(spec.num_samples)
    cfg.dt = float(spec.dt)
    cfg.lam = float(spec.lam)
    L = list(spec.noise_chol) + [0.0] * 36
    for i in range(36):
        cfg.noise_chol[i] = float(L[i])
    for name in ("u_min", "u_max", "goal", "Q", "R", "Qf", "q_limit"):
        v = list(getattr(spec, name))
        arr = getattr(cfg, name)
        for i in range(6):
            arr[i] = float(v[i]) if i < len(v) else 0.0
    cfg.dbscan_eps = float(spec.dbscan_eps)
    cfg.dbscan_min_pts = int(spec.dbscan_min_pts)
    cfg.norm_eps = float(spec.norm_eps)
    cfg.scene_mode = int(spec.scene_mode)
    cfg.history_len = int(spec.history_len)
    cfg.v_obs_min = float(spec.v_obs_min)
    cfg.ref_mode = int(spec.ref_mode)
    cfg.max_obstacles = int(getattr(spec, "max_obstacles", 64))
    cfg.robot_radius = float(spec.robot_radius)
    dh = np.asarray(spec.dh, dtype=np.float32).reshape(6, 4)
    for i in range(6):
        for j in range(4):
            cfg.dh[i][j] = float(dh[i, j])
    cfg.n_link_spheres = int(spec.n_link_spheres)
    cfg.link_sphere_radius = float(spec.link_sphere_radius)
    cfg.w_limit = float(spec.w_limit)
    cfg.seed = int(spec.seed) & 0xFFFFFFFFFFFFFFFF
    cfg.stream_id = int(spec.stream_id) & 0xFFFFFFFF
    cfg.flags = int(getattr(spec, "flags", 0) or 0) & 0xFFFFFFFF
    cfg.device = int(device)
    return cfg


def _dims(dynamics: int):
    return (3, 2, 2) if dynamics == DYN_UNICYCLE else (12, 6, 3)


def _stream_handle(stream) -> int:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Planner:
    """One CE-MPPI planner on a GPU.  Inputs and outputs are torch tensors on
    that GPU; calls are asynchronous on the current (or given) torch stream."""

    def __init__(self, spec, device: int = 0):
        import torch

        self.spec = spec
        self.device = torch.device("cuda", device)
        self.cfg = config_from_spec(spec, device)
        self.n, self.m, self.p = _dims(int(spec.dynamics))
        self.N, self.K = int(spec.horizon), int(spec.num_samples)
        self.handle = ce_mppi_create(self.cfg)
        dev = self.device
        self.u_out = torch.zeros(self.m, dtype=torch.float32, device=dev)
        self.U_out = torch.zeros(self.N, self.m, dtype=torch.float32, device=dev)
        self.info_buf = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)

    @classmethod
    def borrowed(cls, handle: int, spec, device: int = 0) -> "Planner":
        """A view of a planner owned elsewhere (a server session): the same
        calls, but close() leaves the planner alone."""
        import torch

        self = cls.__new__(cls)
        self.spec = spec
        self.device = torch.device("cuda", device)
        self.cfg = config_from_spec(spec, device)
        self.n, self.m, self.p = _dims(int(spec.dynamics))
        self.N, self.K = int(spec.horizon), int(spec.num_samples)
        self.handle = handle
        self._borrowed = True
        dev = self.device
        self.u_out = torch.zeros(self.m, dtype=torch.float32, device=dev)
        self.U_out = torch.zeros(self.N, self.m, dtype=torch.float32, device=dev)
        self.info_buf = torch.zeros(INFO_BYTES, dtype=torch.uint8, device=dev)
        return self

    def close(self):
        if getattr(self, "handle", None):
            if not getattr(self, "_borrowed", False):
                ce_mppi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- state
    def set_nominal(self, U, stream=None):
        import torch

        U = torch.as_tensor(U, dtype=torch.float32).to(self.device).contiguous()
        assert U.shape == (self.N, self.m)
        _check("ce_mppi_set_nominal",
               load().ce_mppi_set_nominal(self.handle, U.data_ptr(), _stream_handle(stream)))
        self._keep = U

    def get_nominal(self, stream=None):
        import torch

        U = torch.empty(self.N, self.m, dtype=torch.float32, device=self.device)
        _check("ce_mppi_get_nominal",
               load().ce_mppi_get_nominal(self.handle, U.data_ptr(), _stream_handle(stream)))
        return U

    def reset_history(self, stream=None):
        _check("ce_mppi_reset_history", load().ce_mppi_reset_history(self.handle, _stream_handle(stream)))

    def set_history(self, hist, stream=None):
        """hist: [h_count][n_obs][p] device tensor of obstacle centres, newest first."""
        import torch

        hist = torch.as_tensor(hist, dtype=torch.float32).to(self.device).contiguous()
        h_count = int(hist.shape[0])
        n_obs = int(hist.shape[1]) if hist.dim() == 3 else 0
        _check("ce_mppi_set_history",
               load().ce_mppi_set_history(self.handle, hist.data_ptr() if hist.numel() else None, h_count,
                                          n_obs, _stream_handle(stream)))

    def set_step(self, step: int, stream=None):
        _check("ce_mppi_set_step", load().ce_mppi_set_step(self.handle, int(step), _stream_handle(stream)))

    def get_state(self, stream=None) -> bytes:
        n = C.c_size_t()
        _check("ce_mppi_state_size", load().ce_mppi_state_size(self.handle, C.byref(n)))
        buf = (C.c_char * n.value)()
        _check("ce_mppi_get_state",
               load().ce_mppi_get_state(self.handle, buf, n.value, _stream_handle(stream)))
        return bytes(buf)

    def set_state(self, state: bytes, stream=None):
        buf = C.create_string_buffer(state, len(state))
        _check("ce_mppi_set_state",
               load().ce_mppi_set_state(self.handle, buf, len(state), _stream_handle(stream)))

    # -- replan
    def replan(self, x_t, obstacles=None, stream=None, want_U: bool = True, want_info: bool = True):
        """x_t: [n] device tensor; obstacles: [n_obs][p+1] device tensor or None.
        Returns (u_out, U_out or None, info buffer or None) as device tensors."""
        n_obs = 0 if obstacles is None else int(obstacles.shape[0])
        obs_ptr = obstacles.data_ptr() if n_obs else None
        ce_mppi_replan(self.handle, x_t.data_ptr(), obs_ptr, n_obs, self.u_out.data_ptr(),
                       self.U_out.data_ptr() if want_U else None,
                       self.info_buf.data_ptr() if want_info else None, _stream_handle(stream))
        return self.u_out, (self.U_out if want_U else None), (self.info_buf if want_info else None)

    def info(self) -> dict:
        """Read the info struct of the last replan (synchronises)."""
        raw = self.info_buf.cpu().numpy().tobytes()
        return CeMppiInfo.from_buffer_copy(raw).as_dict()

    def replan_from_rollouts(self, x_t, obstacles, S, collide, first_obs, p_term, p_first, eps,
                             stream=None):
        n_obs = 0 if obstacles is None else int(obstacles.shape[0])
        _check("ce_mppi_replan_from_rollouts", load().ce_mppi_replan_from_rollouts(
            self.handle, x_t.data_ptr(), obstacles.data_ptr() if n_obs else None, n_obs,
            S.data_ptr(), collide.data_ptr(), first_obs.data_ptr(), p_term.data_ptr(),
            p_first.data_ptr(), eps.data_ptr(), self.u_out.data_ptr(), self.U_out.data_ptr(),
            self.info_buf.data_ptr(), _stream_handle(stream)))
        return self.u_out, self.U_out, self.info_buf

    # -- launch mode and timing
    def set_launch_mode(self, mode: int):
        _check("ce_mppi_set_launch_mode", load().ce_mppi_set_launch_mode(self.handle, int(mode)))

    # -- DBSCAN path
    def set_dbscan_mode(self, mode: int):
        _check("ce_mppi_set_dbscan_mode", load().ce_mppi_set_dbscan_mode(self.handle, int(mode)))

    def dbscan_path(self) -> int:
        v = C.c_int32()
        _check("ce_mppi_get_dbscan_path", load().ce_mppi_get_dbscan_path(self.handle, C.byref(v)))
        return int(v.value)

    def tune_launch(self, x_t, obstacles=None, reps: int = 50, stream=None):
        """Time both launch modes on these inputs and keep the faster;
        returns (us_graph, us_direct) per replan."""
        n_obs = 0 if obstacles is None else int(obstacles.shape[0])
        g, d = C.c_double(), C.c_double()
        _check("ce_mppi_tune_launch", load().ce_mppi_tune_launch(
            self.handle, x_t.data_ptr(), obstacles.data_ptr() if n_obs else None, n_obs,
            self.u_out.data_ptr(), int(reps), _stream_handle(stream), C.byref(g), C.byref(d)))
        return g.value, d.value

    def timing_enable(self, capacity: int):
        _check("ce_mppi_timing_enable", load().ce_mppi_timing_enable(self.handle, int(capacity)))

    def timing_read(self) -> dict:
        r, q, a, n = C.c_double(), C.c_double(), C.c_double(), C.c_int32()
        _check("ce_mppi_timing_read", load().ce_mppi_timing_read(
            self.handle, C.byref(r), C.byref(q), C.byref(a), C.byref(n)))
        return dict(rollout_ms=r.value, post_ms=q.value, total_ms=a.value, count=n.value)

    def timing_read_each(self, cap: int):
        """Per timed replan (rollout_ms, post_ms, total_ms) arrays."""
        r = np.zeros(cap)
        q = np.zeros(cap)
        t = np.zeros(cap)
        n = C.c_int32()
        _check("ce_mppi_timing_read_each",
               load().ce_mppi_timing_read_each(self.handle, int(cap), r.ctypes.data, q.ctypes.data,
                                               t.ctypes.data, C.byref(n)))
        k = min(cap, n.value)
        return r[:k], q[:k], t[:k]

    def time_rollout(self, x_t, obstacles=None, reps: int = 100, stream=None) -> float:
        """Mean ms per launch of the rollout kernel alone (state restored)."""
        n_obs = 0 if obstacles is None else int(obstacles.shape[0])
        ms = C.c_double()
        _check("ce_mppi_time_rollout", load().ce_mppi_time_rollout(
            self.handle, x_t.data_ptr(), obstacles.data_ptr() if n_obs else None, n_obs, int(reps),
            _stream_handle(stream), C.byref(ms)))
        return ms.value

    # -- stages and diagnostics
    def stage_noise(self, step: int, stream=None):
        import torch

        B = (self.N * self.m + 3) // 4
        words = torch.zeros(self.K, B, 4, dtype=torch.int32, device=self.device)
        gauss = torch.zeros(self.K, self.N, self.m, dtype=torch.float32, device=self.device)
        _check("ce_mppi_stage_noise", load().ce_mppi_stage_noise(
            self.handle, int(step) & 0xFFFFFFFF, words.data_ptr(), gauss.data_ptr(),
            _stream_handle(stream)))
        return words, gauss

    def stage_dbscan(self, z, stream=None):
        import torch

        V = int(z.shape[0])
        z = z.to(self.device, torch.float32).contiguous()
        ncount = torch.zeros(max(V, 1), dtype=torch.int32, device=self.device)
        label = torch.zeros(max(V, 1), dtype=torch.int32, device=self.device)
        M = torch.zeros(1, dtype=torch.int32, device=self.device)
        _check("ce_mppi_stage_dbscan", load().ce_mppi_stage_dbscan(
            self.handle, z.data_ptr() if V else None, V, ncount.data_ptr(), label.data_ptr(),
            M.data_ptr(), _stream_handle(stream)))
        return label[:V], ncount[:V], M

    def debug(self, which: int, count: int, dtype=None, cols: Optional[int] = None):
        """Copy an internal buffer of the last replan: `count` rows (x cols)."""
        import torch

        if dtype is None:
            dtype = torch.int32 if which in (DBG_COLLIDE, DBG_FIRST_OBS, DBG_V_IDX, DBG_NCOUNT,
                                             DBG_LABEL, DBG_CLUSTER_SIZE, DBG_TREES) else torch.float32
        shape = (count,) if cols is None else (count, cols)
        out = torch.zeros(shape if count else (1,), dtype=dtype, device=self.device)
        nbytes = out.numel() * out.element_size() if count else 0
        _check("ce_mppi_debug_get", load().ce_mppi_debug_get(self.handle, int(which), out.data_ptr(),
                                                              nbytes, _stream_handle(None)))
        return out[:count] if count else out[:0]


def dbscan_noalloc(z, eps: float, min_pts: int, device: int = 0, stream=None):
    """ce_mppi_dbscan_noalloc on a [V][p] float32 device tensor; returns
    (label, ncount, n_clusters) device tensors (allocated here, by the caller
    of the entry point)."""
    import torch

    z = z.contiguous()
    V, p = int(z.shape[0]), int(z.shape[1])
    dev = torch.device("cuda", device)
    lab = torch.empty(V, dtype=torch.int32, device=dev)
    cnt = torch.empty(V, dtype=torch.int32, device=dev)
    M = torch.empty(1, dtype=torch.int32, device=dev)
    _check("ce_mppi_dbscan_noalloc", load().ce_mppi_dbscan_noalloc(
        int(device), z.data_ptr() if V else None, V, p, float(eps), int(min_pts),
        cnt.data_ptr() if V else None, lab.data_ptr() if V else None, M.data_ptr(),
        _stream_handle(stream)))
    return lab, cnt, M


class Batch:
    """Many planners replanned by one graph launch (``ce_mppi_batch_*``).
    Every member keeps its own buffers; per-call inputs and outputs are torch
    tensors on the members' GPU."""

    def __init__(self, planners):
        self.planners = list(planners)
        arr = (_vp * len(self.planners))(*[p.handle for p in self.planners])
        h = _vp()
        _check("ce_mppi_batch_create",
               load().ce_mppi_batch_create(arr, len(self.planners), C.byref(h)))
        self.handle = h.value
        self._io = (CeMppiBatchIO * len(self.planners))()
        self._keep = None

    def close(self):
        if getattr(self, "handle", None):
            load().ce_mppi_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_io(self, xs, obstacles, want_U: bool = True, want_info: bool = True, u_outs=None):
        """Point the per-call inputs at device tensors (one per member) and the
        outputs at each member planner's own output tensors (or at the given
        u_out tensors)."""
        keep = []
        for i, (pl, x, o) in enumerate(zip(self.planners, xs, obstacles)):
            e = self._io[i]
            n_obs = 0 if o is None else int(o.shape[0])
            e.x_t = x.data_ptr()
            e.obstacles = o.data_ptr() if n_obs else None
            e.n_obs = n_obs
            e.reserved = 0
            e.u_out = (u_outs[i] if u_outs is not None else pl.u_out).data_ptr()
            e.U_out = pl.U_out.data_ptr() if want_U else None
            e.info = pl.info_buf.data_ptr() if want_info else None
            keep.append((x, o))
        self._keep = (keep, u_outs)

    def replan(self, stream=None):
        _check("ce_mppi_batch_replan",
               load().ce_mppi_batch_replan(self.handle, self._io, _stream_handle(stream)))

    def replan_subset(self, members, stream=None):
        """Replan only the listed members (indices into the planner list) with
        the inputs and outputs last given to ``set_io``."""
        members = [int(m) for m in members]
        idx = (C.c_int32 * len(members))(*members)
        # out-of-range members are passed through for the library to reject
        io = (CeMppiBatchIO * len(members))(
            *[self._io[m] if 0 <= m < len(self._io) else CeMppiBatchIO() for m in members])
        _check("ce_mppi_batch_replan_subset",
               load().ce_mppi_batch_replan_subset(self.handle, idx, len(members), io,
                                                  _stream_handle(stream)))

    def set_tuning(self, colg: int, tile_blocks_per_cu: int, roll_blocks_per_cu: int,
                   roll_per_wave: int = 4):
        t = CeMppiBatchTuning(int(colg), int(tile_blocks_per_cu), int(roll_blocks_per_cu),
                              int(roll_per_wave))
        _check("ce_mppi_batch_set_tuning", load().ce_mppi_batch_set_tuning(self.handle, C.byref(t)))

    def get_tuning(self) -> dict:
        t = CeMppiBatchTuning()
        _check("ce_mppi_batch_get_tuning", load().ce_mppi_batch_get_tuning(self.handle, C.byref(t)))
        return t.as_dict()

    def autotune(self, reps: int = 3, stream=None):
        t = CeMppiBatchTuning()
        ms = C.c_double()
        _check("ce_mppi_batch_autotune",
               load().ce_mppi_batch_autotune(self.handle, self._io, int(reps), _stream_handle(stream),
                                             C.byref(t), C.byref(ms)))
        return t.as_dict(), ms.value


class Server:
    """Continuous-batching replan server over resident sessions
    (``ce_mppi_server_*``).  Inputs and outputs are host numpy arrays."""

    def __init__(self, device: int = 0, max_batch: int = 256, max_inflight: int = 3,
                 memory_budget: int = 0, mode: int = 0):
        """mode: SERVE_BATCHED (continuous batching) or SERVE_PLAIN (one request
        at a time through ce_mppi_replan; max_batch = max_inflight = 1)."""
        cfg = CeMppiServerConfig(int(device), int(max_batch), int(max_inflight), int(mode),
                                 int(memory_budget))
        h = _vp()
        _check("ce_mppi_server_create", load().ce_mppi_server_create(C.byref(cfg), C.byref(h)))
        self.handle = h.value
        self.device = int(device)
        self.dims = []

    def open_session(self, spec, U0=None) -> int:
        cfg = config_from_spec(spec, self.device)
        sid = C.c_int32()
        U = None if U0 is None else np.ascontiguousarray(U0, dtype=np.float32)
        _check("ce_mppi_server_open_session",
               load().ce_mppi_server_open_session(self.handle, C.byref(cfg),
                                                  U.ctypes.data if U is not None else None,
                                                  C.byref(sid)))
        self.dims.append(_dims(int(spec.dynamics)))
        return sid.value

    def start(self):
        _check("ce_mppi_server_start", load().ce_mppi_server_start(self.handle))

    def submit(self, session: int, x_t, obstacles) -> int:
        x = np.ascontiguousarray(x_t, dtype=np.float32)
        o = np.ascontiguousarray(obstacles, dtype=np.float32)
        t = C.c_uint64()
        _check("ce_mppi_server_submit",
               load().ce_mppi_server_submit(self.handle, int(session), x.ctypes.data,
                                            o.ctypes.data if len(o) else None, len(o), C.byref(t)))
        return t.value

    def wait(self, ticket: int, session: int):
        n, m, p = self.dims[session]
        u = np.zeros(m, np.float32)
        info = CeMppiInfo()
        lat = C.c_double()
        _check("ce_mppi_server_wait",
               load().ce_mppi_server_wait(self.handle, int(ticket), u.ctypes.data, C.byref(info),
                                          C.byref(lat)))
        return u, info.as_dict(), lat.value

    def run_trace(self, t_arrival, sessions, x, obstacles, n_obs):
        """Replay a request trace: arrays t_arrival [n] (s), sessions [n],
        x [n][12], obstacles [n][256] (rows of p+1 floats packed), n_obs [n].
        Returns (latency_s [n], u_out [n][6])."""
        n = len(t_arrival)
        t = np.ascontiguousarray(t_arrival, dtype=np.float64)
        sess = np.ascontiguousarray(sessions, dtype=np.int32)
        xs = np.ascontiguousarray(x, dtype=np.float32)
        ob = np.ascontiguousarray(obstacles, dtype=np.float32)
        no = np.ascontiguousarray(n_obs, dtype=np.int32)
        lat = np.zeros(n, np.float64)
        u = np.zeros((n, 6), np.float32)
        _check("ce_mppi_server_run_trace",
               load().ce_mppi_server_run_trace(self.handle, n, t.ctypes.data, sess.ctypes.data,
                                               xs.ctypes.data, ob.ctypes.data, no.ctypes.data,
                                               lat.ctypes.data, u.ctypes.data))
        return lat, u

    def session_planner(self, session: int, spec) -> "Planner":
        """The planner of a session (owned by the server) as a Planner view."""
        h = load().ce_mppi_server_session_planner(self.handle, int(session))
        if not h:
            raise CeMppiError("ce_mppi_server_session_planner", CE_EINVAL, "unknown session")
        return Planner.borrowed(h, spec, self.device)

    def stats(self) -> dict:
        st = CeMppiServerStats()
        _check("ce_mppi_server_get_stats", load().ce_mppi_server_get_stats(self.handle, C.byref(st)))
        return st.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            load().ce_mppi_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

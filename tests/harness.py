"""Shared helpers of the GPU parity tests: run the HIP planner through the
C-ABI binding and collect its buffers as numpy arrays; tolerance helpers."""
from __future__ import annotations

import numpy as np

from paper_2607_06499_amd import binding as B

# Tolerances.  FP32 kernels against the FP64 oracle on the same noise: a
# horizon of N <= 63 steps accumulates O(N) FP32 roundings (about 6e-8
# each) in the states and O(N) more in the cost sums, well under 1e-4
# relative; the Gaussians come from hardware log/sqrt/sin/cos with a
# measured worst case of 3.2e-7 against FP64, under 2e-6.
TRAJ_RTOL = 1e-4        # trajectories, costs: |d| <= 1e-4 * max(|ref|, 1)
GAUSS_TOL = 2e-6        # standard normals: |d| <= 2e-6 * max(|g|, 1)
BOUNDARY = 2e-5         # rollouts within 2e-5 (relative) of a contact boundary are flagged
PAIR_BAND = 1e-4        # feature pairs within 1e-4 * eps of eps are flagged


def torch_mod():
    import torch

    return torch


def gpu_ok() -> bool:
    try:
        import torch

        return torch.cuda.is_available()
    except Exception:
        return False


def to_dev(a, dtype=None):
    torch = torch_mod()
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda").contiguous()


def collect(pl: "B.Planner", info: dict) -> dict:
    """Read back the per-rollout and per-cluster buffers of the last replan."""
    torch = torch_mod()
    torch.cuda.synchronize()
    K, p, N, m = pl.K, pl.p, pl.N, pl.m
    out = dict(info=info)
    out["S"] = pl.debug(B.DBG_COST, K).cpu().numpy()
    out["col"] = pl.debug(B.DBG_COLLIDE, K).cpu().numpy()
    out["first_obs"] = pl.debug(B.DBG_FIRST_OBS, K).cpu().numpy()
    out["p_term"] = pl.debug(B.DBG_P_TERM, K, cols=p).cpu().numpy()
    out["p_first"] = pl.debug(B.DBG_P_FIRST, K, cols=p).cpu().numpy()
    out["eps_eff"] = pl.debug(B.DBG_EPS, K * N * m).cpu().numpy().reshape(K, N, m)
    V = info["n_feasible"] if info["branch"] == 0 else 0
    out["v_idx"] = pl.debug(B.DBG_V_IDX, V).cpu().numpy()
    out["z"] = pl.debug(B.DBG_Z, V, cols=p).cpu().numpy()
    out["g"] = pl.debug(B.DBG_G, V, cols=p).cpu().numpy()
    out["ncount"] = pl.debug(B.DBG_NCOUNT, V).cpu().numpy()
    out["label"] = pl.debug(B.DBG_LABEL, V).cpu().numpy()
    M = info["n_clusters"] if info["branch"] == 0 else 0
    out["c_mean_cost"] = pl.debug(B.DBG_CLUSTER_COST, M).cpu().numpy()
    out["c_dir"] = pl.debug(B.DBG_CLUSTER_DIR, M, cols=p).cpu().numpy()
    out["c_size"] = pl.debug(B.DBG_CLUSTER_SIZE, M).cpu().numpy()
    torch.cuda.synchronize()
    return out


def gpu_replan(pl: "B.Planner", x_t, obs) -> dict:
    torch = torch_mod()
    x = to_dev(np.asarray(x_t, np.float32))
    o = to_dev(np.asarray(obs, np.float32)) if len(obs) else None
    u, U, _ = pl.replan(x, o)
    torch.cuda.synchronize()
    info = pl.info()
    r = collect(pl, info)
    r["u_out"] = u.cpu().numpy().copy()
    r["U_new"] = U.cpu().numpy().copy()
    r["U_next"] = pl.get_nominal().cpu().numpy().copy()
    return r


def rel_err(a, b, floor=1.0):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def feature_slack(p_term, ref, floor: float = 2e-5, rel: float = 1e-6):
    """Per-point bound on |z_gpu - z_oracle| for z = d / |d|, d = p_term - ref:
    a perturbation delta of d moves z by at most 2 |delta| / |d|, and the FP32
    path perturbs d by about rel * (|p_term| + |ref| + 1)."""
    p_term = np.asarray(p_term, np.float64)
    ref = np.asarray(ref, np.float64)
    dn = np.linalg.norm(p_term - ref[None, :], axis=1)
    mag = np.linalg.norm(p_term, axis=1) + np.linalg.norm(ref) + 1.0
    return floor + 2.0 * rel * mag / np.maximum(dn, 1e-9)


def flagged_pairs(z, eps: float, band: float = PAIR_BAND, slack=None):
    """Indices of points in a pair whose distance is within band*eps of eps
    (plus the two points' feature slack, when given)."""
    z = np.asarray(z, np.float64)
    if len(z) < 2:
        return np.zeros(0, int), 0
    d = np.sqrt(((z[:, None, :] - z[None, :, :]) ** 2).sum(-1))
    lim = band * eps
    if slack is not None:
        sl = np.asarray(slack, np.float64)
        lim = lim + sl[:, None] + sl[None, :]
    near = np.abs(d - eps) <= lim
    np.fill_diagonal(near, False)
    pts = np.nonzero(near.any(1))[0]
    return pts, int(near.sum() // 2)


def canonical_partition(labels):
    groups = {}
    for i, l in enumerate(labels):
        if l >= 0:
            groups.setdefault(int(l), []).append(i)
    return sorted(tuple(g) for g in groups.values())


def counts_agree(gpu, exact, min_pts: int) -> bool:
    """Neighbour counts as the kernels report them: a count scan stops once
    a point is known to be core, so the count is exact below minPts and lies
    between minPts and the exact count for core points."""
    gpu = np.asarray(gpu)
    exact = np.asarray(exact)
    low = exact < min_pts
    return bool(np.array_equal(gpu[low], exact[low])
                and np.all(gpu[~low] >= min_pts) and np.all(gpu[~low] <= exact[~low]))

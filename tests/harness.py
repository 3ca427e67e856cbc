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
    pl.replan(x, o)
    torch.cuda.synchronize()
    return collect_outputs(pl)


def collect_outputs(pl: "B.Planner", info: dict = None, u_out=None) -> dict:
    """Buffers and outputs of the planner's last replan (by ce_mppi_replan or
    a batch replan into the planner's own output tensors).  With u_out and
    info given (a served request), U_new is rebuilt from u_out and the kept,
    shifted sequence."""
    torch = torch_mod()
    torch.cuda.synchronize()
    own = info is None
    if own:
        info = pl.info()
    r = collect(pl, info)
    r["U_next"] = pl.get_nominal().cpu().numpy().copy()
    if own:
        r["u_out"] = pl.u_out.cpu().numpy().copy()
        r["U_new"] = pl.U_out.cpu().numpy().copy()
    else:
        r["u_out"] = np.asarray(u_out, np.float32).copy()
        r["U_new"] = np.concatenate([r["u_out"][None, :], r["U_next"][:-1]], axis=0)
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


def feature_slack_measured(pT_gpu, pT_orc, ref_gpu, ref_orc):
    """Per-point bound on |z_gpu - z_oracle| from the measured differences of
    the inputs of Eq. (13): z = d / |d| moves by at most 2 |delta| / |d| when d
    moves by delta, and the FP32 path adds the rounding of d = p - ref (one
    ulp of each operand) and of the normalisation (a few ulps of z)."""
    u = 2.0 ** -24
    pg = np.asarray(pT_gpu, np.float64)
    po = np.asarray(pT_orc, np.float64)
    rg = np.asarray(ref_gpu, np.float64)[None, :]
    ro = np.asarray(ref_orc, np.float64)[None, :]
    d = np.linalg.norm(po - ro, axis=1)
    delta = (np.linalg.norm(pg - po, axis=1) + np.linalg.norm(rg - ro, axis=1)
             + 2.0 * u * (np.linalg.norm(po, axis=1) + np.linalg.norm(ro, axis=1)))
    return 2.0 * delta / np.maximum(d, 1e-12) + 8.0 * u


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


# Flagged-pair band when the GPU and the oracle cluster the same FP32
# features: the kernels form d^2 = fma(dy, dy, dx * dx) from FP32 operands,
# three roundings of relative size u = 2^-24 each, and compare it with the
# rounded eps^2 (one more), so |d_fp32 - d_exact| <= 2.5 u d + u eps/2 ~
# 2e-7 eps near the boundary; 1e-6 eps leaves a factor of five.
STAGE_BAND = 1e-6


def _pair_blocks(z, block=512):
    V = len(z)
    sq = (z * z).sum(1)
    for r0 in range(0, V, block):
        r1 = min(V, r0 + block)
        d2 = sq[r0:r1, None] + sq[None, :] - 2.0 * (z[r0:r1] @ z.T)
        # the expansion loses digits for close pairs: recompute those directly
        near = d2 < 4.0 * 1e-6 + 1e-300
        if near.any():
            ri, ci = np.nonzero(near)
            d2[ri, ci] = ((z[r0 + ri] - z[ci]) ** 2).sum(1)
        yield r0, r1, np.sqrt(np.maximum(d2, 0.0))


def dbscan_check(z, eps: float, min_pts: int, gpu_count, gpu_label, half_lim, exact_ref=None,
                 tag: str = ""):
    """Check a GPU DBSCAN result on features z (taken as FP64) against the
    definition (closed eps-ball, minPts counts the point itself, border point
    -> cluster of its lowest-index core neighbour, clusters numbered by their
    lowest core index), leaving free every pair whose distance lies within
    half_lim[k] + half_lim[l] of eps (the flagged pairs).

    Asserts that the GPU result is exactly DBSCAN of some neighbour graph that
    agrees with the exact one on every unflagged pair: neighbour counts
    (exact below minPts, between minPts and the count for core points), core
    flags, the partition of the core points, the border rule and the
    canonical numbering.  With no flagged pair the labels must equal
    exact_ref (the oracle's labels on the same features) if it is given.
    Returns the numbers of flagged pairs, flagged points and points whose
    label differs from exact_ref."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components

    z = np.asarray(z, np.float64)
    V = len(z)
    cnt = np.asarray(gpu_count, np.int64)
    lab = np.asarray(gpu_label, np.int64)
    assert cnt.shape == (V,) and lab.shape == (V,), tag
    if V == 0:
        return dict(flagged_pairs=0, flagged_points=0, differing=0)
    hl = np.broadcast_to(np.asarray(half_lim, np.float64), (V,))
    core = cnt >= min_pts
    cnt_lo = np.zeros(V, np.int64)
    cnt_fl = np.zeros(V, np.int64)
    low_sure = np.full(V, V, np.int64)      # lowest-index surely-adjacent GPU core point
    fl_rows, fl_cols = [], []
    comp = np.arange(V)
    for r0, r1, D in _pair_blocks(z):
        rows = np.arange(r0, r1)
        lim = hl[rows, None] + hl[None, :]
        flag = np.abs(D - eps) <= lim
        sure = (D <= eps) & ~flag
        flag[rows - r0, rows] = False
        sure[rows - r0, rows] = True
        cnt_lo[r0:r1] = sure.sum(1)
        cnt_fl[r0:r1] = flag.sum(1)
        fr, fc = np.nonzero(flag)
        fl_rows.append(fr + r0)
        fl_cols.append(fc)
        sc = sure & core[None, :]
        has = sc.any(1)
        low_sure[r0:r1] = np.where(has, sc.argmax(1), V)
        # no surely-adjacent pair of GPU core points may sit in two clusters
        cross = sc & core[rows, None] & (lab[None, :] != lab[rows, None])
        assert not cross.any(), f"{tag}: adjacent core points in different clusters"
        # connectivity inside each cluster over sure and flagged edges
        ri, ci = np.nonzero((sure | flag) & core[rows, None] & core[None, :]
                            & (lab[None, :] == lab[rows, None]))
        a, b = comp[ri + r0], comp[ci]
        keep = a != b
        if keep.any():
            key = np.unique(a[keep] * V + b[keep])
            g = coo_matrix((np.ones(len(key)), (key // V, key % V)), shape=(V, V))
            _, cc = connected_components(g, directed=False)
            comp = cc[comp]
    fr = np.concatenate(fl_rows)
    fc = np.concatenate(fl_cols)
    n_flag_pairs = int(len(fr) // 2)
    flagged_pts = np.zeros(V, bool)
    flagged_pts[fr] = True
    cnt_hi = cnt_lo + cnt_fl
    # counts and core flags
    low = cnt < min_pts
    assert np.all((cnt_lo[low] <= cnt[low]) & (cnt[low] <= cnt_hi[low])), f"{tag}: neighbour counts"
    assert np.all(cnt_hi[~low] >= cnt[~low]), f"{tag}: core counts"
    sure_core = cnt_lo >= min_pts
    sure_non = cnt_hi < min_pts
    assert np.all(core[sure_core]) and not np.any(core[sure_non]), f"{tag}: core flags"
    # core points carry labels; each cluster is connected and numbered canonically
    assert np.all(lab[core] >= 0), f"{tag}: unlabelled core point"
    M = int(lab.max()) + 1 if np.any(lab >= 0) else 0
    assert np.all(lab >= -1), tag
    firsts = []
    for c in range(M):
        members = np.nonzero(core & (lab == c))[0]
        assert len(members), f"{tag}: cluster {c} without core points"
        assert len(np.unique(comp[members])) == 1, f"{tag}: cluster {c} not connected"
        firsts.append(members[0])
    assert firsts == sorted(firsts), f"{tag}: clusters not numbered by their lowest core index"
    # border and noise points
    fl_core = {}
    for a, b in zip(fr, fc):
        if core[b] and not core[a]:
            fl_core.setdefault(int(a), []).append(int(b))
    for k in np.nonzero(~core)[0]:
        L = int(low_sure[k])
        allowed = {int(lab[L])} if L < V else {-1}
        for f in fl_core.get(int(k), []):
            if f < L:
                allowed.add(int(lab[f]))
        assert int(lab[k]) in allowed, f"{tag}: border point {k} label {lab[k]} not in {allowed}"
    differing = 0
    if exact_ref is not None:
        ref = np.asarray(exact_ref, np.int64)
        differing = int(np.sum(ref != lab))
        if n_flag_pairs == 0:
            assert differing == 0, f"{tag}: labels differ with no flagged pair"
    return dict(flagged_pairs=n_flag_pairs, flagged_points=int(flagged_pts.sum()), differing=differing)

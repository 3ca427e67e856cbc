#!/usr/bin/env python3
"""CE-MPPI replan benchmark on one MI355X.

Workload (default): the dynamic 2-D scene -- unicycle, K=8192 rollouts,
horizon N=50, dt=0.05 s, 24 moving circular obstacles in a 20x20 m box,
dynamic selection rule, DBSCAN eps=0.25 / minPts=20 -- driven through a
closed loop of 50 + 400 replans.  The loop is recorded first (untimed, host
plant), its inputs uploaded to the GPU; a step is then one replay of the
400-replan segment from the planner state it started from (the state restore
included), so every step holds the loop's clustering and fallback replans in
their natural mix.  Inputs are resident in HBM when the timed region starts,
and the replays reproduce the recorded loop bit for bit.

Prints one JSON line: replans/s (value), rollout-steps/s, p50/p99 latency,
per-branch latency and device time, the roofline of the rollout kernel and
the CPU oracle baseline (one thread and every host core).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CE-MPPI replans/s + rollout-steps/s at K=8192; p50/p99 replan latency"
# MI355X FP32 vector: 256 CUs x 2.4 GHz x 64 lanes x 2 (FMA) = 78.6 TFLOP/s
# without packed FP32 instructions (this build disables them); the datasheet's
# 157.3 TFLOP/s counts the packed (two-wide) FMA
PEAK_FP32_TFLOPS = 78.6
PEAK_FP32_PACKED_TFLOPS = 157.3
N_CU, CLOCK_HZ = 256, 2.4e9
PEAK_HBM_GBS = 8000.0
LOOP_WARM, LOOP_LEN = 50, 400


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed steps: replays of the recorded closed-loop segment")
    ap.add_argument("--warmup", type=int, default=2, help="untimed replays before them")
    ap.add_argument("--loop", type=int, default=LOOP_LEN, help="replans per replay (the timed segment)")
    ap.add_argument("--loop-warm", type=int, default=LOOP_WARM,
                    help="closed-loop replans recorded before the timed segment")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workload", default="unicycle_dynamic", type=_workload_name,
                    help="unicycle_dynamic, unicycle_dynamic_ahead, unicycle_static, "
                         "unicycle_static_ahead, arm6_dynamic, unicycle_dynamic_cv, arm6_pose, "
                         "batch_uneven or served_sessions; a single-planner workload may take "
                         "another rollout count as <name>@<K>")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="budget of each CPU-oracle baseline sample (one thread, then every core)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the clustering-branch companion measurement")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-form companion measurement")
    ap.add_argument("--no-scaling", action="store_true",
                    help="skip the clustering-branch replays at K = 16384 and 65536")
    ap.add_argument("--no-companions", action="store_true",
                    help="skip the static 2-D and arm workloads")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served-form measurement")
    ap.add_argument("--batch-steps", type=int, default=30,
                    help="timed batch steps of the batched-form measurement")
    ap.add_argument("--rollout-reps", type=int, default=2000,
                    help="back-to-back rollout launches timed for the roofline")
    ap.add_argument("--dbscan", default="auto", choices=["auto", "window", "bitmap", "tiled"],
                    help="DBSCAN path of the single-planner workloads (auto: the planner's default)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (profiler calibration)")
    return ap.parse_args()


SINGLE_WORKLOADS = ("unicycle_dynamic", "unicycle_dynamic_ahead", "unicycle_static",
                    "unicycle_static_ahead", "arm6_dynamic", "unicycle_dynamic_cv", "arm6_pose")


def _workload_name(s):
    base, _, k = s.partition("@")
    ok = (s in ("batch_uneven", "served_sessions") or
          (base in SINGLE_WORKLOADS and (not k or (k.isdigit() and 1 <= int(k) <= 65536))))
    if not ok:
        raise argparse.ArgumentTypeError(f"unknown workload {s!r}")
    return s


def scene_for(name, seed):
    from paper_2607_06499_amd import workloads as W

    table = {"unicycle_dynamic": W.unicycle_dynamic,
             "unicycle_dynamic_ahead": W.unicycle_dynamic_ahead,
             "unicycle_static": W.unicycle_static,
             "unicycle_static_ahead": W.unicycle_static_ahead,
             "arm6_dynamic": W.arm6_dynamic,
             "unicycle_dynamic_cv": W.unicycle_dynamic_cv,
             "arm6_pose": W.arm6_pose}
    if "@" in name:
        # another rollout count: "<workload>@<K>"
        base, k = name.split("@")
        return table[base](seed, num_samples=int(k))
    return table[name](seed)


def record_loop(pl, scene, T, torch, snap_at=0):
    """Run the closed loop for T replans (host plant), returning the inputs
    each replan saw, the applied controls, the per-replan info and the
    planner state before replan snap_at."""
    from paper_2607_06499_amd import plant
    from paper_2607_06499_amd.binding import DBG_TREES

    spec = scene.spec
    fld = scene.field.copy()
    x = scene.x0.astype(np.float64)
    X, OBS, UO, INFO = [], [], [], []
    snap = None
    xd = torch.zeros(spec.n, dtype=torch.float32, device="cuda")
    od = torch.zeros(max(fld.n, 1), spec.p + 1, dtype=torch.float32, device="cuda")
    for t in range(T):
        if t == snap_at:
            snap = pl.get_state()
        xf = np.asarray(x, np.float32)
        obs = fld.observation()
        X.append(xf)
        OBS.append(obs)
        xd.copy_(torch.from_numpy(xf))
        od[: fld.n].copy_(torch.from_numpy(obs))
        u, _, _ = pl.replan(xd, od[: fld.n])
        torch.cuda.synchronize()
        info = pl.info()
        if info["branch"] == 0:
            info["trees"], info["tree_fallback"] = pl.debug(DBG_TREES, 2).cpu().tolist()
        un = u.cpu().numpy().copy()
        UO.append(un)
        INFO.append(info)
        x = plant.step(spec.dynamics, x, un, spec.dt)
        fld.step(spec.dt)
    return np.stack(X), np.stack(OBS), np.stack(UO), INFO, snap


def timed_passes(pl, lib, Xd, Od, n_obs, t0, L, snap, W, K, torch):
    """W untimed and K timed replays of the L recorded replans from t0, each
    from the planner state snap (the restore is inside the timed region)."""
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    h = pl.handle
    u_ptr = pl.u_out.data_ptr()
    xs = [Xd[t].data_ptr() for t in range(t0, t0 + L)]
    os_ = [Od[t].data_ptr() for t in range(t0, t0 + L)]
    f = lib.ce_mppi_replan

    def one_pass():
        pl.set_state(snap)
        for t in range(L):
            f(h, xs[t], os_[t], n_obs, u_ptr, None, None, sh)

    for _ in range(W):
        one_pass()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t_start = time.perf_counter()
    e0.record(stream)
    for _ in range(K):
        one_pass()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    return wall, e0.elapsed_time(e1) / 1e3


def latency_replay(pl, lib, Xd, Od, n_obs, t0, L, snap, torch, Uo):
    """One replan at a time, host wall clock from the call to u_out ready, and
    a bit-for-bit check against the recorded loop."""
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    h = pl.handle
    f = lib.ce_mppi_replan
    pl.set_state(snap)
    lat = []
    outs = torch.zeros(L, pl.m, dtype=torch.float32, device="cuda")
    for t in range(L):
        ts = time.perf_counter()
        f(h, Xd[t0 + t].data_ptr(), Od[t0 + t].data_ptr(), n_obs, outs[t].data_ptr(), None, None, sh)
        stream.synchronize()
        lat.append(time.perf_counter() - ts)
    same = bool(np.array_equal(outs.cpu().numpy(), Uo[t0: t0 + L]))
    return np.array(lat), same


def device_times(pl, lib, Xd, Od, n_obs, t0, L, snap, torch):
    """Per replan of the segment: device time of the rollout kernel, of the
    rest and of the whole replan (HIP events around direct launches)."""
    pl.set_state(snap)
    pl.timing_enable(L)
    sh = int(torch.cuda.current_stream().cuda_stream)
    for t in range(t0, t0 + L):
        lib.ce_mppi_replan(pl.handle, Xd[t].data_ptr(), Od[t].data_ptr(), n_obs, pl.u_out.data_ptr(),
                           None, None, sh)
    torch.cuda.synchronize()
    r, q, a = pl.timing_read_each(L)
    pl.timing_enable(0)
    return r, q, a


def copy_calibration(torch, mib: int, reps: int = 5):
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters of a profiler run: reads and writes exactly mib MiB each."""
    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()


def source_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_record(name, kernel_sources):
    """A committed counter summary (profiles/<name>), if it was taken on the
    current kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_digest") != source_digest(kernel_sources):
        return None
    return rec


def _oracle_worker(args):
    """Oracle replans of the recorded loop from its start (its own nominal
    sequence), one after another, until the budget is spent: (count, s)."""
    spec, U0, X, OBS, hist_len, budget_s, start_evt = args
    import oracle

    oracle.load()
    if start_evt is not None:
        start_evt.wait()
    U = np.asarray(U0, np.float64)
    hist = []
    n = 0
    t0 = time.perf_counter()
    for t in range(len(X)):
        hist.insert(0, OBS[t][:, : spec.p].astype(np.float64))
        hist = hist[:hist_len]
        r = oracle.replan(spec, X[t], U, OBS[t], np.array(hist), step=t)
        U = r["U_next"]
        n += 1
        if time.perf_counter() - t0 >= budget_s and n >= 2:
            break
    return n, time.perf_counter() - t0


def _pool_worker(args):
    return _oracle_worker(args)


def host_cpu():
    """Host CPU model and the cores this process may use (the box's share)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail, os.cpu_count() or avail


def cpu_baseline(scene, X, OBS, budget_s, hist_len, max_workers=16):
    """The FP64 C oracle as it stands on this host: one thread, then one
    worker process per core (up to the box's share), every worker replaying
    the same closed loop; the rate is the sum of the workers' rates while
    they run together."""
    spec = scene.spec
    model, avail, total = host_cpu()
    n1, t1 = _oracle_worker((spec, scene.U0, X, OBS, hist_len, budget_s, None))
    cores = max(1, min(avail, max_workers))
    ctx = mp.get_context("spawn")
    with ctx.Manager() as mgr:
        evt = mgr.Event()
        with ctx.Pool(cores) as pool:
            res = pool.map_async(_pool_worker, [(spec, scene.U0, X, OBS, hist_len, budget_s, evt)] * cores)
            time.sleep(1.0)  # let the workers import and load the oracle
            evt.set()
            out = res.get()
    rate_all = sum(n / dt for n, dt in out)
    steps = spec.num_samples * spec.horizon
    return dict(value=round(rate_all, 3), unit="replans/s", cores=cores, kind="oracle",
                sample=f"the recorded closed loop (K={spec.num_samples}, N={spec.horizon}) replayed from "
                       f"its start by the single-threaded FP64 C oracle in {cores} worker processes "
                       f"for about {budget_s:g} s each ({sum(n for n, _ in out)} replans in all)",
                one_thread=dict(value=round(n1 / t1, 3), unit="replans/s", cores=1, replans=n1,
                                rollout_steps_per_s=round(steps * n1 / t1, 1)),
                rollout_steps_per_s=round(steps * rate_all, 1),
                host={"cpu_model": model, "cores_available": avail, "cores_total": total})


def live_obstacles(spec, x, obs):
    """Obstacles the unicycle rollout kernel keeps after its exact broad phase
    (frozen obstacles): every state lies within max|v| N dt of p(x_t), so an
    obstacle whose surface is farther (plus a margin) is never tested."""
    if spec.dynamics != 0:
        return len(obs)
    vmax = max(abs(float(spec.u_min[0])), abs(float(spec.u_max[0])))
    if not np.isfinite(vmax):
        return len(obs)
    reach = vmax * spec.horizon * float(spec.dt)
    d = np.hypot(obs[:, 0] - x[0], obs[:, 1] - x[1])
    ext = reach + float(spec.robot_radius) + obs[:, 2]
    return int(np.sum(d <= ext + 1e-3 * ext + 1e-3))


def rollout_flops(spec, n_obs):
    """Algorithmic FP32 flops of one rollout launch with n_obs obstacles
    tested: 25 + 5 n_obs per unicycle rollout-step (noise transform 6, clamp
    4, dynamics 6, cost 9, 5 per obstacle test); forward kinematics 480, link
    spheres 48, 8 per sphere-obstacle test and 40 for noise and cost per arm
    rollout-step.  Constant-velocity obstacles add the displacement of each
    tested obstacle (4 flops in 2-D, 6 in 3-D); the pose cost adds 62 per arm
    rollout-step (orientation error 60, distance 2)."""
    steps = spec.num_samples * spec.horizon
    cv = bool(getattr(spec, "flags", 0) & 2)
    pose = bool(getattr(spec, "flags", 0) & 1)
    if spec.dynamics == 0:
        return steps * (25 + (9 if cv else 5) * n_obs)
    return steps * (480 + 48 + (14 if cv else 8) * n_obs * spec.n_link_spheres + 40 + (62 if pose else 0))


def _ms(a):
    return round(float(a) * 1e3, 4)


DBSCAN_NAMES = {1: "window", 2: "bitmap", 3: "tiled"}


def run_workload(name, seed, loop_warm, L, W, K, torch, B, want_timing=True, rollout_reps=2000,
                 dbscan_mode=0):
    scene = scene_for(name, seed)
    spec = scene.spec
    lib = B.load()
    pl = B.Planner(spec)
    pl.set_dbscan_mode(dbscan_mode)
    dbscan_path = DBSCAN_NAMES[pl.dbscan_path()]
    pl.set_nominal(torch.as_tensor(scene.U0).cuda())
    X, OBS, Uo, INFO, snap = record_loop(pl, scene, loop_warm + L, torch, snap_at=loop_warm)
    Xd = torch.as_tensor(X).cuda()
    Od = torch.as_tensor(OBS).cuda()
    n_obs = OBS.shape[1]
    t0 = loop_warm
    # throughput, in both launch modes (graph replay, direct launches): which
    # one is faster depends on the host of this box; the faster is reported
    walls = {}
    for mode, code in (("graph", B.LAUNCH_GRAPH), ("direct", B.LAUNCH_DIRECT)):
        pl.set_launch_mode(code)
        walls[mode] = timed_passes(pl, lib, Xd, Od, n_obs, t0, L, snap, W, K, torch)
    best = min(walls, key=lambda m: walls[m][0])
    wall, gpu = walls[best]
    pl.set_launch_mode(B.LAUNCH_GRAPH if best == "graph" else B.LAUNCH_DIRECT)
    launch = {"mode": best, "us_per_replan_graph": round(1e6 * walls["graph"][0] / (K * L), 2),
              "us_per_replan_direct": round(1e6 * walls["direct"][0] / (K * L), 2)}
    lat, same = latency_replay(pl, lib, Xd, Od, n_obs, t0, L, snap, torch, Uo)
    dev = device_times(pl, lib, Xd, Od, n_obs, t0, L, snap, torch) if want_timing else None
    kernel_ms = None
    if want_timing:
        # the rollout kernel alone, back to back on the replan stream, on the
        # first timed replan's inputs (the planner state is restored after)
        pl.set_state(snap)
        kernel_ms = pl.time_rollout(Xd[t0], Od[t0], reps=rollout_reps)
    info = INFO[t0: t0 + L]
    branches = np.array([i["branch"] for i in info])
    mix = {"cluster": int(np.sum(branches == 0)), "fallback": int(np.sum(branches == 1)),
           "all_collide": int(np.sum(branches == 2))}
    per_branch = {}
    for bname, code in (("cluster", 0), ("fallback", 1), ("all_collide", 2)):
        sel = branches == code
        if not sel.any():
            continue
        e = {"replans": int(sel.sum()),
             "latency_ms": {"p50": _ms(np.percentile(lat[sel], 50)), "p99": _ms(np.percentile(lat[sel], 99)),
                            "mean": _ms(np.mean(lat[sel]))}}
        if dev is not None:
            e["device_us"] = {"rollout": round(float(np.mean(dev[0][sel])) * 1e3, 2),
                              "after_rollout": round(float(np.mean(dev[1][sel])) * 1e3, 2),
                              "replan": round(float(np.mean(dev[2][sel])) * 1e3, 2)}
        if code == 0:
            e["mean_feasible"] = round(float(np.mean([i["n_feasible"] for i, b in zip(info, branches) if b == 0])), 1)
        per_branch[bname] = e
    trees = [i["trees"] for i in info if i["branch"] == 0]
    tstat = {"mean": round(float(np.mean(trees)), 1) if trees else 0.0,
             "max": int(max(trees)) if trees else 0,
             "union_find_fallback": int(sum(i["tree_fallback"] for i in info if i["branch"] == 0))}
    n_live = live_obstacles(spec, X[t0], OBS[t0])
    pl.close()
    return dict(scene=scene, X=X, OBS=OBS, wall=wall, gpu=gpu, lat=lat, same=same, launch=launch,
                kernel_ms=kernel_ms, mix=mix, per_branch=per_branch, trees=tstat, n_live=n_live,
                L=L, K=K, W=W, loop_warm=loop_warm, dbscan_path=dbscan_path)


def companion(name, seed, loop_warm, L, K, torch, B, label):
    """Throughput, latency and rollout roofline of another single-planner
    workload (same protocol as the headline: K replays of an L-replan loop)."""
    r = run_workload(name, seed, loop_warm, L, 1, K, torch, B, rollout_reps=500)
    spec = r["scene"].spec
    flops = rollout_flops(spec, r["n_live"])
    rate = K * L / r["wall"]
    return {
        "workload": label, "replans_per_s": round(rate, 1),
        "rollout_steps_per_s": round(rate * spec.num_samples * spec.horizon, 1),
        "latency_ms": {"p50": _ms(np.percentile(r["lat"], 50)), "p99": _ms(np.percentile(r["lat"], 99))},
        "branch_mix": r["mix"], "per_branch": r["per_branch"], "replay_bit_exact": r["same"],
        "launch": r["launch"], "rollout_kernel_ms": round(r["kernel_ms"], 5),
        "obstacles_tested": r["n_live"],
        "rollout_tflops": round(flops / (r["kernel_ms"] * 1e-3) / 1e12, 4),
    }


def run_batch(seed, W, K, torch, B, autotune=True, n_planners=256):
    """Batched form on the uneven 256-planner workload: a closed loop is
    recorded with the batch (host plant between steps), then replayed from
    the same initial states twice, as one batch graph launch per step and as
    one plain replan per planner per step (graph replay each), on the same
    device-resident inputs.  Returns throughput, step latency and whether the
    two replays agree bitwise."""
    from paper_2607_06499_amd import plant
    from paper_2607_06499_amd import workloads as WL

    members = WL.batch_uneven(seed, n_planners)
    scenes = [m.scene for m in members]
    n = len(scenes)
    pls = [B.Planner(s.spec) for s in scenes]
    for sc, pl in zip(scenes, pls):
        pl.set_nominal(torch.as_tensor(sc.U0).cuda())
    states0 = [pl.get_state() for pl in pls]
    batch = B.Batch(pls)
    T = W + K
    dev = "cuda"
    xdev = torch.zeros(T, n, 3, dtype=torch.float32, device=dev)
    odev = [torch.zeros(T, max(sc.field.n, 1), 3, dtype=torch.float32, device=dev) for sc in scenes]
    nobs = [sc.field.n for sc in scenes]
    U = torch.zeros(T, n, 2, dtype=torch.float32, device=dev)
    rows = lambda t: [U[t, i] for i in range(n)]
    fields = [sc.field.copy() for sc in scenes]
    xs = [sc.x0.astype(np.float64) for sc in scenes]
    tune = None
    # record
    for t in range(T):
        xdev[t].copy_(torch.from_numpy(np.asarray(xs, np.float32)))
        for i, f in enumerate(fields):
            if nobs[i]:
                odev[i][t, : nobs[i]].copy_(torch.from_numpy(f.observation()))
        batch.set_io([xdev[t, i] for i in range(n)],
                     [odev[i][t, : nobs[i]] if nobs[i] else None for i in range(n)],
                     want_U=False, want_info=False, u_outs=rows(t))
        if t == 0 and autotune:
            tune, _ = batch.autotune(reps=3)
        batch.replan()
        u = U[t].cpu().numpy().astype(np.float64)
        for i in range(n):
            xs[i] = plant.step(0, xs[i], u[i], scenes[i].spec.dt)
            fields[i].step(scenes[i].spec.dt)
    U_rec = U.cpu().numpy().copy()
    io = []
    for t in range(T):
        batch.set_io([xdev[t, i] for i in range(n)],
                     [odev[i][t, : nobs[i]] if nobs[i] else None for i in range(n)],
                     want_U=False, want_info=False, u_outs=rows(t))
        io.append((B.CeMppiBatchIO * n).from_buffer_copy(batch._io))
    lib = B.load()
    stream = int(torch.cuda.current_stream().cuda_stream)

    def batch_pass(sync_each):
        for pl, st in zip(pls, states0):
            pl.set_state(st)
        U.zero_()
        lat = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(T):
            if t == W:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            t1 = time.perf_counter()
            B._check("ce_mppi_batch_replan", lib.ce_mppi_batch_replan(batch.handle, io[t], stream))
            if sync_each:
                torch.cuda.synchronize()
                if t >= W:
                    lat.append(time.perf_counter() - t1)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, np.array(lat)

    wall_b, _ = batch_pass(False)
    same_b = bool(np.array_equal(U.cpu().numpy(), U_rec))
    _, lat_b = batch_pass(True)
    # the same steps as plain replans, one planner after another, in each
    # launch mode (the faster one is the plain form's number on this machine)
    handles = [pl.handle for pl in pls]

    def sequential_pass(mode):
        for pl, st in zip(pls, states0):
            pl.set_state(st)
            pl.set_launch_mode(mode)
        U.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(T):
            if t == W:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
            for i in range(n):
                e = io[t][i]
                lib.ce_mppi_replan(handles[i], e.x_t, e.obstacles, e.n_obs, e.u_out, None, None, stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, bool(np.array_equal(U.cpu().numpy(), U_rec))

    wall_g, same_g = sequential_pass(B.LAUNCH_GRAPH)
    wall_d, same_d = sequential_pass(B.LAUNCH_DIRECT)
    seq_mode = "direct" if wall_d < wall_g else "graph"
    wall_s = min(wall_g, wall_d)
    same_s = same_g and same_d
    Ks = np.array([sc.spec.num_samples for sc in scenes])
    Ns = np.array([sc.spec.horizon for sc in scenes])
    batch.close()
    for pl in pls:
        pl.close()
    return {
        "workload": f"batch_uneven: {n} unicycle planners, K log-uniform [256,16384] "
                    f"(sum {int(Ks.sum())}), N uniform [20,60], 4..64 obstacles, half static "
                    f"half dynamic, closed loop of {T} steps (seed {seed})",
        "replans_per_s": round(n * K / wall_b, 1),
        "ms_per_batch_step": round(1e3 * wall_b / K, 4),
        "rollout_steps_per_s": round(float((Ks * Ns).sum()) * K / wall_b, 1),
        "latency_ms": {"p50": round(float(np.percentile(lat_b, 50)) * 1e3, 4),
                       "p99": round(float(np.percentile(lat_b, 99)) * 1e3, 4)},
        "sequential_plain": {"replans_per_s": round(n * K / wall_s, 1),
                             "ms_per_round": round(1e3 * wall_s / K, 4), "launch": seq_mode,
                             "ms_per_round_graph": round(1e3 * wall_g / K, 4),
                             "ms_per_round_direct": round(1e3 * wall_d / K, 4)},
        "speedup_vs_sequential": round(wall_s / wall_b, 3),
        "tuning": tune,
        "bitwise_equal_to_recorded_loop": {"batched": same_b, "sequential": same_s},
    }


def run_serve(seed, torch, B, rates=(2000.0, 5000.0, 10000.0, 20000.0), seconds=0.75):
    """Served form: 512 resident sessions, Poisson-arrival replan requests at
    each rate through the continuous-batching server and through the plain
    form (one request at a time, each through ce_mppi_replan of its session:
    the single-planner kernels in the launch mode tuned per session), on the
    same trace.  Latency is request arrival to completion."""
    from paper_2607_06499_amd import workloads as WL

    sess = WL.served_sessions(seed)
    scenes = [s.scene for s in sess]

    def make(max_batch, max_inflight, mode):
        srv = B.Server(max_batch=max_batch, max_inflight=max_inflight, mode=mode)
        for sc in scenes:
            srv.open_session(sc.spec, sc.U0)
        srv.start()
        return srv

    out = {"workload": f"served_sessions: {len(scenes)} sessions "
                       f"({sum(s.kind == 'unicycle' for s in sess)} unicycle K log-uniform "
                       f"[1024,8192], {sum(s.kind == 'arm' for s in sess)} arm K log-uniform "
                       f"[1024,4096]), Poisson arrivals, sessions drawn uniformly (seed {seed})",
           "rates": []}
    for rate in rates:
        n = int(rate * seconds)
        t, sid = WL.poisson_arrivals(rate, n, len(scenes), seed)
        x = np.zeros((n, 12), np.float32)
        ob = np.zeros((n, 256), np.float32)
        no = np.zeros(n, np.int32)
        for i, k in enumerate(sid):
            sc = scenes[k]
            x[i, : len(sc.x0)] = sc.x0
            o = np.asarray(sc.obstacles, np.float32)
            no[i] = len(o)
            ob[i, : o.size] = o.ravel()
        row = {"offered_req_per_s": rate, "requests": n}
        for name, mb, fl, mode in (("continuous_batching", 256, 3, B.SERVE_BATCHED),
                                   ("plain_one_per_launch", 1, 1, B.SERVE_PLAIN)):
            srv = make(mb, fl, mode)
            t0 = time.perf_counter()
            lat, _ = srv.run_trace(t, sid, x, ob, no)
            wall = time.perf_counter() - t0
            st = srv.stats()
            srv.close()
            row[name] = {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
                         "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
                         "replans_per_s": round(n / wall, 1),
                         "mean_batch": round(st["mean_batch"], 2), "launches": st["launches"]}
        out["rates"].append(row)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU: the CE-MPPI planners are "
                                   "independent, so more GPUs would each run their own share of "
                                   "planners with no data crossing between them; run with --gpus 1"}))
        sys.exit(2)
    import torch

    from paper_2607_06499_amd import binding as B

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    W, K = args.warmup, args.steps
    if args.workload == "served_sessions":
        rs = run_serve(args.seed, torch, B)
        top = rs["rates"][-1]["continuous_batching"]
        print(json.dumps({"metric": "CE-MPPI served replans/s and p50/p99 latency (continuous batching, "
                                    "512 sessions, Poisson arrivals)", "value": top["replans_per_s"],
                          "unit": "replans/s", "n_gpus": 1, "steps": rs["rates"][-1]["requests"],
                          "warmup": 0, "ms_per_step": round(1e3 / top["replans_per_s"], 5),
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                          "dtype": "f32", "data": "synthetic", "config": {"workload": rs["workload"]},
                          "rates": rs["rates"]}))
        return
    if args.workload == "batch_uneven":
        rb = run_batch(args.seed, min(W, 5), args.batch_steps, torch, B)
        print(json.dumps({"metric": "CE-MPPI replans/s, batched form (256 uneven planners per "
                                    "graph launch)", "value": rb["replans_per_s"], "unit": "replans/s",
                          "n_gpus": 1, "steps": args.batch_steps, "warmup": min(W, 5),
                          "ms_per_step": rb["ms_per_batch_step"], "higher_is_better": True,
                          "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                          "config": {"workload": rb["workload"]}, **{k: v for k, v in rb.items()
                                                                     if k != "workload"}}))
        return
    dmode = {"auto": 0, "window": 1, "bitmap": 2, "tiled": 3}[args.dbscan]
    res = run_workload(args.workload, args.seed, args.loop_warm, args.loop, W, K, torch, B,
                       rollout_reps=args.rollout_reps, dbscan_mode=dmode)
    if args.calibrate_copy_mib:
        copy_calibration(torch, args.calibrate_copy_mib)
    spec = res["scene"].spec
    L = args.loop
    replans_per_s = K * L / res["wall"]
    rollout_steps = spec.num_samples * spec.horizon
    lat = res["lat"]
    # roofline of the rollout kernel on the first timed replan's inputs:
    # algorithmic flops with the obstacles the exact broad phase keeps
    n_obs = res["OBS"].shape[1]
    flops = rollout_flops(spec, res["n_live"])
    t_roll = res["kernel_ms"] * 1e-3
    achieved = flops / t_roll / 1e12
    ksrc = [os.path.join(ROOT, "paper_2607_06499_amd", "csrc", f)
            for f in ("rollout.hip", "device.hpp")]
    traffic_rec = profile_record("rollout_unicycle_k8192_n50_traffic.json", ksrc)
    valu_rec = profile_record("rollout_unicycle_k8192_n50_valu.json", ksrc)
    roofline = {
        "bound": "alu", "kernel": "rollout",
        "achieved": round(achieved, 4), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved / PEAK_FP32_TFLOPS, 6),
        "traffic": traffic_rec.get("hbm_bytes_per_launch") if traffic_rec else None,
        "kernel_ms": round(t_roll * 1e3, 5),
        "algorithmic_flop_per_launch": flops,
        "obstacles_tested": res["n_live"], "obstacles": n_obs,
        "peak_note": "FP32 vector without packed instructions (disabled in this build); "
                     f"the packed datasheet peak is {PEAK_FP32_PACKED_TFLOPS}",
        "frac_of_packed_peak": round(achieved / PEAK_FP32_PACKED_TFLOPS, 6),
    }
    if valu_rec:
        # executed FP32 work and VALU issue from the committed counter run
        # at the live kernel time: the issue ceiling is one wave64 VALU
        # instruction per CU per cycle (four 16-lane SIMDs, four cycles each)
        cf = valu_rec["fp32_flop_per_launch"]
        vi = valu_rec["valu_insts_per_launch"]
        roofline["counters"] = {
            "fp32_flop_per_launch": cf,
            "fp32_tflops_at_kernel_ms": round(cf / t_roll / 1e12, 4),
            "fp32_frac_of_peak": round(cf / t_roll / 1e12 / PEAK_FP32_TFLOPS, 4),
            "valu_insts_per_launch": vi,
            "valu_issue_utilisation": round(vi / (N_CU * CLOCK_HZ * t_roll), 4),
            "fp32_share_of_valu": valu_rec["fp32_share_of_valu"],
            "source": "profiles/rollout_unicycle_k8192_n50_valu.json",
        }
    out = {
        "metric": METRIC,
        "value": round(replans_per_s, 2),
        "unit": "replans/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(1e3 * res["wall"] / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: unicycle K={spec.num_samples} N={spec.horizon} "
                         f"dt={spec.dt:g} {n_obs} moving obstacles, "
                         f"{'dynamic' if spec.scene_mode else 'static'} rule, closed loop of "
                         f"{args.loop_warm} + {L} replans (seed {args.seed}); a step replays the "
                         f"{L}-replan segment")
            if spec.dynamics == 0 else
            f"{args.workload}: 6-joint arm K={spec.num_samples} N={spec.horizon} {n_obs} spheres; "
            f"a step replays {L} closed-loop replans",
            "K": spec.num_samples, "N": spec.horizon, "n_obs": n_obs, "replans_per_step": L,
            "branch_mix": res["mix"],
            "dbscan_path": res["dbscan_path"],
            "dbscan_trees": res["trees"],
            "launch": res["launch"],
        },
        "rollout_steps_per_s": round(replans_per_s * rollout_steps, 1),
        "latency_ms": {"p50": _ms(np.percentile(lat, 50)), "p99": _ms(np.percentile(lat, 99))},
        "per_branch": res["per_branch"],
        "gpu_ms_per_step": round(1e3 * res["gpu"] / K, 4),
        "replay_bit_exact": res["same"],
        "roofline": roofline,
    }
    if not args.no_probe and args.workload == "unicycle_dynamic":
        pr = run_workload("unicycle_dynamic_ahead", args.seed, 0, 40, 1, max(K, 5), torch, B,
                          dbscan_mode=dmode)
        out["clustering_branch"] = {
            "workload": "unicycle_dynamic_ahead: same planner, obstacle ahead in the robot's path "
                        "(replays of a 40-replan loop)",
            "replans_per_s": round(pr["K"] * pr["L"] / pr["wall"], 2),
            "latency_ms": {"p50": _ms(np.percentile(pr["lat"], 50)), "p99": _ms(np.percentile(pr["lat"], 99))},
            "branch_mix": pr["mix"], "per_branch": pr["per_branch"], "dbscan_path": pr["dbscan_path"],
            "dbscan_trees": pr["trees"],
        }
        # the same loop on the other single-planner DBSCAN paths (same bits)
        ab = {}
        for m in (1, 2, 3):
            if DBSCAN_NAMES[m] == pr["dbscan_path"]:
                continue
            q = run_workload("unicycle_dynamic_ahead", args.seed, 0, 40, 1, max(K, 5), torch, B,
                             want_timing=True, rollout_reps=20, dbscan_mode=m)
            ab[q["dbscan_path"]] = {"replans_per_s": round(q["K"] * q["L"] / q["wall"], 2),
                                    "device_us": q["per_branch"]["cluster"].get("device_us")}
        out["clustering_branch"]["other_dbscan_paths"] = ab
        # the same scene with more rollouts: the pairwise paths grow with
        # V^2, the window path with V (the bitmap stops at K = 16384)
        if not args.no_scaling:
            scal = {}
            for ks, modes in ((16384, (1, 2, 3)), (65536, (1, 3))):
                sc = {}
                for m in modes:
                    q = run_workload(f"unicycle_dynamic_ahead@{ks}", args.seed, 0, 20, 1, 3, torch, B,
                                     want_timing=True, rollout_reps=20, dbscan_mode=m)
                    cb = q["per_branch"].get("cluster", {})
                    sc[q["dbscan_path"]] = {"replans_per_s": round(q["K"] * q["L"] / q["wall"], 2),
                                            "branch_mix": q["mix"],
                                            "mean_feasible": cb.get("mean_feasible"),
                                            "device_us": cb.get("device_us")}
                scal[f"K{ks}"] = sc
            out["clustering_branch"]["larger_K"] = dict(
                workload="unicycle_dynamic_ahead with K=16384 and K=65536 rollouts (replays of a "
                         "20-replan loop) on each single-planner DBSCAN path", **scal)
    if not args.no_companions and args.workload == "unicycle_dynamic":
        cK = max(2, min(K, 3))
        out["static_2d"] = companion("unicycle_static", args.seed, 0, 200, cK, torch, B,
                                     "unicycle_static: K=1024 N=30 dt=0.1, 8 static obstacles, "
                                     "replays of a 200-replan closed loop")
        out["static_2d_ahead"] = companion("unicycle_static_ahead", args.seed, 0, 200, cK, torch, B,
                                           "unicycle_static_ahead: obstacle 1.2 m ahead, replays of a "
                                           "200-replan closed loop")
        out["arm_6dof"] = companion("arm6_dynamic", args.seed, 0, 400, cK, torch, B,
                                    "arm6_dynamic: K=4096 N=32 dt=0.05, 16 moving spheres, "
                                    "8 link spheres, replays of a 400-replan closed loop")
        out["dynamic_2d_const_vel"] = companion(
            "unicycle_dynamic_cv", args.seed, args.loop_warm, L, cK, torch, B,
            "unicycle_dynamic_cv: the headline scene with constant-velocity obstacle prediction "
            "inside the rollouts")
        out["arm_6dof_pose"] = companion(
            "arm6_pose", args.seed, 0, 400, cK, torch, B,
            "arm6_pose: arm6_dynamic with the real-robot pose cost (10, 3, 1000) and "
            "constant-velocity obstacles, replays of a 400-replan closed loop")
    if not args.no_batch and args.workload == "unicycle_dynamic":
        out["batched_form"] = run_batch(args.seed, 5, args.batch_steps, torch, B)
    if not args.no_serve and args.workload == "unicycle_dynamic":
        out["served_form"] = run_serve(args.seed, torch, B)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(res["scene"], res["X"], res["OBS"], args.cpu_seconds,
                                           spec.history_len)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

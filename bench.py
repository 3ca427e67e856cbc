#!/usr/bin/env python3
"""CE-MPPI replan benchmark on one MI355X.

Workload (default): the dynamic 2-D scene -- unicycle, K=8192 rollouts,
horizon N=50, dt=0.05 s, 24 moving circular obstacles in a 20x20 m box,
dynamic selection rule, DBSCAN eps=0.25 / minPts=20 -- driven through a
closed loop.  A step is one replan (the whole hot path).  The loop's states
and observations are recorded first (untimed), uploaded to the GPU, and the
planner (reset to its initial state) then replans over them back to back:
inputs are resident in HBM when the timed region starts, and the timed
replans reproduce the recorded loop bit for bit.

Prints one JSON line: replans/s (value), rollout-steps/s, p50/p99 latency,
the branch mix, the roofline of the rollout kernel and the CPU oracle
baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CE-MPPI replans/s + rollout-steps/s at K=8192; p50/p99 replan latency"
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (datasheet)
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workload", default="unicycle_dynamic",
                    choices=["unicycle_dynamic", "unicycle_dynamic_ahead", "unicycle_static",
                             "unicycle_static_ahead", "arm6_dynamic", "unicycle_dynamic_cv",
                             "arm6_pose", "batch_uneven", "served_sessions"])
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget of the CPU-oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the clustering-branch companion measurement")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-form companion measurement")
    ap.add_argument("--no-companions", action="store_true",
                    help="skip the static 2-D and arm workloads")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served-form measurement")
    ap.add_argument("--batch-steps", type=int, default=30,
                    help="timed batch steps of the batched-form measurement")
    ap.add_argument("--rollout-reps", type=int, default=2000,
                    help="back-to-back rollout launches timed for the roofline")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (profiler calibration)")
    return ap.parse_args()


def scene_for(name, seed):
    from paper_2607_06499_amd import workloads as W

    return {"unicycle_dynamic": W.unicycle_dynamic,
            "unicycle_dynamic_ahead": W.unicycle_dynamic_ahead,
            "unicycle_static": W.unicycle_static,
            "unicycle_static_ahead": W.unicycle_static_ahead,
            "arm6_dynamic": W.arm6_dynamic,
            "unicycle_dynamic_cv": W.unicycle_dynamic_cv,
            "arm6_pose": W.arm6_pose}[name](seed)


def record_loop(pl, scene, T, torch):
    """Run the closed loop for T replans (host plant), returning the inputs
    each replan saw, the applied controls and the per-replan info."""
    from paper_2607_06499_amd import plant
    from paper_2607_06499_amd.binding import DBG_TREES

    spec = scene.spec
    fld = scene.field.copy()
    x = scene.x0.astype(np.float64)
    X, OBS, UO, INFO = [], [], [], []
    xd = torch.zeros(spec.n, dtype=torch.float32, device="cuda")
    od = torch.zeros(max(fld.n, 1), spec.p + 1, dtype=torch.float32, device="cuda")
    for _ in range(T):
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
    return np.stack(X), np.stack(OBS), np.stack(UO), INFO


def timed_replays(pl, lib, Xd, Od, n_obs, W, K, torch):
    """Back-to-back replans over the recorded inputs: W warm-up, K timed."""
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    h = pl.handle
    u_ptr = pl.u_out.data_ptr()
    xs = [Xd[t].data_ptr() for t in range(W + K)]
    os_ = [Od[t].data_ptr() for t in range(W + K)]
    f = lib.ce_mppi_replan
    for t in range(W):
        f(h, xs[t], os_[t], n_obs, u_ptr, None, None, sh)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for t in range(W, W + K):
        f(h, xs[t], os_[t], n_obs, u_ptr, None, None, sh)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1) / 1e3


def latency_replays(pl, lib, Xd, Od, n_obs, W, K, torch, Uo):
    """One replan at a time, host wall clock from the call to u_out ready."""
    stream = torch.cuda.current_stream()
    sh = int(stream.cuda_stream)
    h = pl.handle
    f = lib.ce_mppi_replan
    lat = []
    outs = torch.zeros(W + K, pl.m, dtype=torch.float32, device="cuda")
    for t in range(W + K):
        t0 = time.perf_counter()
        f(h, Xd[t].data_ptr(), Od[t].data_ptr(), n_obs, outs[t].data_ptr(), None, None, sh)
        stream.synchronize()
        if t >= W:
            lat.append(time.perf_counter() - t0)
    same = bool(np.array_equal(outs.cpu().numpy(), Uo[: W + K]))
    return np.array(lat), same


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


def traffic_record(kernel_sources):
    """HBM traffic per launch from the committed counter summary, if it was
    taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "rollout_unicycle_k8192_n50_traffic.json")
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    if rec.get("source_digest") != source_digest(kernel_sources):
        return None, rec
    return rec.get("hbm_bytes_per_launch"), rec


def cpu_baseline(scene, X, OBS, W, budget_s, hist_len):
    import oracle

    spec = scene.spec
    U = scene.U0.astype(np.float64)
    hist = []
    n = 0
    t0 = time.perf_counter()
    # the oracle replays the same loop from its start (its own nominal
    # sequence), one replan after another, until the budget is spent
    for t in range(len(X)):
        hist.insert(0, OBS[t][:, : spec.p].astype(np.float64))
        hist = hist[:hist_len]
        r = oracle.replan(spec, X[t], U, OBS[t], np.array(hist), step=t)
        U = r["U_next"]
        n += 1
        if time.perf_counter() - t0 >= budget_s and n >= 2:
            break
    dt = time.perf_counter() - t0
    return dict(value=n / dt, unit="replans/s", cores=1, kind="oracle",
                sample=f"first {n} replans of the same closed loop (K={spec.num_samples}, "
                       f"N={spec.horizon}), single-threaded FP64 C oracle, "
                       f"{spec.num_samples * spec.horizon * n / dt:.3g} rollout-steps/s")


def run_workload(name, seed, W, K, torch, B, want_timing=True, rollout_reps=2000):
    scene = scene_for(name, seed)
    spec = scene.spec
    lib = B.load()
    pl = B.Planner(spec)
    pl.set_nominal(torch.as_tensor(scene.U0).cuda())
    state0 = pl.get_state()
    X, OBS, Uo, INFO = record_loop(pl, scene, W + K, torch)
    Xd = torch.as_tensor(X).cuda()
    Od = torch.as_tensor(OBS).cuda()
    n_obs = OBS.shape[1]
    # throughput, in both launch modes (graph replay, direct launches): which
    # one is faster depends on the host of this box; the faster is reported
    walls = {}
    for mode, code in (("graph", B.LAUNCH_GRAPH), ("direct", B.LAUNCH_DIRECT)):
        pl.set_launch_mode(code)
        pl.set_state(state0)
        walls[mode] = timed_replays(pl, lib, Xd, Od, n_obs, W, K, torch)
    best = min(walls, key=lambda m: walls[m][0])
    wall, gpu = walls[best]
    pl.set_launch_mode(B.LAUNCH_GRAPH if best == "graph" else B.LAUNCH_DIRECT)
    launch = {"mode": best, "us_per_replan_graph": round(1e6 * walls["graph"][0] / K, 2),
              "us_per_replan_direct": round(1e6 * walls["direct"][0] / K, 2)}
    # latency (and a bit-for-bit replay check)
    pl.set_state(state0)
    lat, same = latency_replays(pl, lib, Xd, Od, n_obs, W, K, torch, Uo)
    timing = None
    kernel_ms = None
    if want_timing:
        # the rollout kernel alone, back to back on the replan stream, on the
        # first timed replan's inputs (the planner state is restored after)
        pl.set_state(state0)
        kernel_ms = pl.time_rollout(Xd[W], Od[W], reps=rollout_reps)
        pl.set_state(state0)
        pl.timing_enable(W + K)
        for t in range(W + K):
            lib.ce_mppi_replan(pl.handle, Xd[t].data_ptr(), Od[t].data_ptr(), n_obs,
                               pl.u_out.data_ptr(), None, None, int(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        timing = pl.timing_read()
        timing["count"] = max(timing["count"], 1)
        pl.timing_enable(0)
    branches = [i["branch"] for i in INFO[W:]]
    mix = {"cluster": branches.count(0), "fallback": branches.count(1),
           "all_collide": branches.count(2)}
    ncl = [i["n_feasible"] for i in INFO[W:] if i["branch"] == 0]
    trees = [i["trees"] for i in INFO[W:] if i["branch"] == 0]
    tstat = {"mean": round(float(np.mean(trees)), 1) if trees else 0.0,
             "max": int(max(trees)) if trees else 0,
             "union_find_fallback": int(sum(i["tree_fallback"] for i in INFO[W:] if i["branch"] == 0))}
    pl.close()
    return dict(scene=scene, X=X, OBS=OBS, wall=wall, gpu=gpu, lat=lat, same=same, timing=timing, launch=launch,
                kernel_ms=kernel_ms, mix=mix, mean_V=float(np.mean(ncl)) if ncl else 0.0, trees=tstat)


def rollout_flops(spec, n_obs):
    """Algorithmic FP32 flops of one rollout launch: 25 + 5 n_obs per
    unicycle rollout-step (noise transform, clamp, dynamics, cost, 5 per
    obstacle test); forward kinematics 480, link spheres 48, 8 per
    sphere-obstacle test and 40 for noise and cost per arm rollout-step.
    Constant-velocity obstacles add the displacement of each tested obstacle
    (4 flops in 2-D, 6 in 3-D); the pose cost adds 62 per arm rollout-step
    (orientation error 60, distance 2)."""
    steps = spec.num_samples * spec.horizon
    cv = bool(getattr(spec, "flags", 0) & 2)
    pose = bool(getattr(spec, "flags", 0) & 1)
    if spec.dynamics == 0:
        return steps * (25 + (9 if cv else 5) * n_obs)
    return steps * (480 + 48 + (14 if cv else 8) * n_obs * spec.n_link_spheres + 40 + (62 if pose else 0))


def companion(name, seed, W, K, torch, B, label):
    """Throughput, latency and rollout roofline of another single-planner
    workload (same protocol as the headline)."""
    r = run_workload(name, seed, W, K, torch, B, rollout_reps=500)
    spec = r["scene"].spec
    n_obs = r["OBS"].shape[1]
    flops = rollout_flops(spec, n_obs)
    return {
        "workload": label, "replans_per_s": round(K / r["wall"], 1),
        "rollout_steps_per_s": round(K / r["wall"] * spec.num_samples * spec.horizon, 1),
        "latency_ms": {"p50": round(float(np.percentile(r["lat"], 50)) * 1e3, 4),
                       "p99": round(float(np.percentile(r["lat"], 99)) * 1e3, 4)},
        "branch_mix": r["mix"], "replay_bit_exact": r["same"], "launch": r["launch"],
        "rollout_kernel_ms": round(r["kernel_ms"], 5),
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
    form (one request per launch, one launch at a time), on the same trace.
    Latency is request arrival to completion."""
    from paper_2607_06499_amd import workloads as WL

    sess = WL.served_sessions(seed)
    scenes = [s.scene for s in sess]

    def make(max_batch, max_inflight):
        srv = B.Server(max_batch=max_batch, max_inflight=max_inflight)
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
        for name, mb, fl in (("continuous_batching", 256, 3), ("plain_one_per_launch", 1, 1)):
            srv = make(mb, fl)
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
    res = run_workload(args.workload, args.seed, W, K, torch, B, rollout_reps=args.rollout_reps)
    if args.calibrate_copy_mib:
        copy_calibration(torch, args.calibrate_copy_mib)
    spec = res["scene"].spec
    replans_per_s = K / res["wall"]
    rollout_steps = spec.num_samples * spec.horizon
    lat = res["lat"]
    # roofline of the rollout kernel: algorithmic FP32 flops per rollout-step
    # 25 + 5 n_obs (noise transform, clamp, dynamics, cost, 5 per obstacle)
    n_obs = res["OBS"].shape[1]
    flops = rollout_flops(spec, n_obs)
    t_roll = res["kernel_ms"] * 1e-3
    t_roll_launch = res["timing"]["rollout_ms"] / res["timing"]["count"] * 1e-3
    achieved = flops / t_roll / 1e12
    ksrc = [os.path.join(ROOT, "paper_2607_06499_amd", "csrc", f)
            for f in ("rollout.hip", "device.hpp")]
    traffic, _ = traffic_record(ksrc)
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
            "workload": f"{args.workload}: unicycle K={spec.num_samples} N={spec.horizon} "
                        f"dt={spec.dt:g} {n_obs} obstacles, "
                        f"{'dynamic' if spec.scene_mode else 'static'} rule, "
                        f"closed loop of {W + K} replans (seed {args.seed})"
            if spec.dynamics == 0 else
            f"{args.workload}: 6-joint arm K={spec.num_samples} N={spec.horizon} {n_obs} spheres",
            "K": spec.num_samples, "N": spec.horizon, "n_obs": n_obs,
            "branch_mix": res["mix"], "mean_feasible_when_clustering": round(res["mean_V"], 1),
            "dbscan_trees": res["trees"],
            "launch": res["launch"],
        },
        "rollout_steps_per_s": round(replans_per_s * rollout_steps, 1),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 4),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 4)},
        "gpu_ms_per_step": round(1e3 * res["gpu"] / K, 4),
        "replay_bit_exact": res["same"],
        "roofline": {
            "bound": "alu", "kernel": "rollout",
            "achieved": round(achieved, 4), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 6),
            "traffic": traffic,
            "kernel_ms": round(t_roll * 1e3, 5),
            "kernel_ms_in_replan_with_launch": round(t_roll_launch * 1e3, 5),
            "algorithmic_flop_per_launch": flops,
        },
    }
    if not args.no_probe and args.workload == "unicycle_dynamic":
        pr = run_workload("unicycle_dynamic_ahead", args.seed, W, K, torch, B, want_timing=False)
        out["clustering_branch"] = {
            "workload": "unicycle_dynamic_ahead: same planner, obstacle ahead in the robot's path",
            "replans_per_s": round(K / pr["wall"], 2),
            "latency_ms": {"p50": round(float(np.percentile(pr["lat"], 50)) * 1e3, 4),
                           "p99": round(float(np.percentile(pr["lat"], 99)) * 1e3, 4)},
            "branch_mix": pr["mix"], "mean_feasible": round(pr["mean_V"], 1),
            "dbscan_trees": pr["trees"],
        }
    if not args.no_companions and args.workload == "unicycle_dynamic":
        out["static_2d"] = companion("unicycle_static", args.seed, W, 200, torch, B,
                                     "unicycle_static: K=1024 N=30 dt=0.1, 8 static obstacles, "
                                     "closed loop of 200 timed replans")
        out["static_2d_ahead"] = companion("unicycle_static_ahead", args.seed, W, 200, torch, B,
                                           "unicycle_static_ahead: obstacle 1.2 m ahead, clustering "
                                           "branch")
        out["arm_6dof"] = companion("arm6_dynamic", args.seed, W, K, torch, B,
                                    "arm6_dynamic: K=4096 N=32 dt=0.05, 16 moving spheres, "
                                    "8 link spheres, closed loop")
        out["dynamic_2d_const_vel"] = companion(
            "unicycle_dynamic_cv", args.seed, W, K, torch, B,
            "unicycle_dynamic_cv: the headline scene with constant-velocity obstacle prediction "
            "inside the rollouts")
        out["arm_6dof_pose"] = companion(
            "arm6_pose", args.seed, W, K, torch, B,
            "arm6_pose: arm6_dynamic with the real-robot pose cost (10, 3, 1000) and "
            "constant-velocity obstacles")
    if not args.no_batch and args.workload == "unicycle_dynamic":
        out["batched_form"] = run_batch(args.seed, 5, args.batch_steps, torch, B)
    if not args.no_serve and args.workload == "unicycle_dynamic":
        out["served_form"] = run_serve(args.seed, torch, B)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(res["scene"], res["X"], res["OBS"], W, args.cpu_seconds,
                                           spec.history_len)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""The angular-window DBSCAN path (single planner, 2-D features) against the
eps-adjacency bitmap and the tiled distance passes on the same inputs, and
against the definition (the oracle's brute-force DBSCAN in FP64).

All three paths decide each pair with the same FP32 distance test, so the
window path must reproduce the bitmap's exact counts and every path's labels
bit for bit; the tiled passes stop counting at minPts, so their counts are
compared by that contract.  The feature sets put the windows' edge cases in
reach: gaps between runs of core buckets swept across the critical angle in
quarter-bucket steps (the boundary tests that link or split runs), clusters
across the +-pi seam, features off the unit ring, duplicates, small and
large eps, a full 16,384-point arc, and planners of 32,768 and 65,536
rollouts, beyond the bitmap's limit."""
import math

import numpy as np
import pytest

import oracle
from paper_2607_06499_amd import workloads as W
from paper_2607_06499_amd.plant import unicycle_step
from tests import harness as H

pytestmark = pytest.mark.gpu

NB = 4096  # angular buckets of the window path


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not H.gpu_ok():
        pytest.skip("no GPU")
    from paper_2607_06499_amd import binding

    binding.load()


def _ring(rng, th, lo=1.0 - 2e-5, hi=1.0 - 1e-7):
    """Points at angles th with norms just below one, as unit features of
    displacements between a few centimetres and some metres have."""
    s = rng.uniform(lo, hi, len(th))
    return (np.stack([np.cos(th), np.sin(th)], 1) * s[:, None]).astype(np.float32)


def _cases():
    rng = np.random.default_rng(7)
    cases = []
    cases.append(("arc_16384", _ring(rng, rng.normal(0.7, 0.35, 16384)), 0.25, 20))
    cases.append(("uniform_3000", _ring(rng, rng.uniform(-math.pi, math.pi, 3000)), 0.1, 5))
    # three arcs whose gaps sweep the critical angle 2 asin(eps / 2)
    eps = 0.25
    crit = 2 * math.asin(eps / 2)
    beta = 2 * math.pi / NB
    for i, phi in enumerate(np.linspace(crit - 3 * beta, crit + 3 * beta, 13)):
        a = np.linspace(-0.5, 0.0, 150)
        b = np.linspace(phi, phi + 0.5, 150)
        c = np.linspace(phi + 0.5 + phi * 1.0001, 2 * phi + 1.0, 150)
        th = np.concatenate([a, b, c]) + rng.uniform(-math.pi, math.pi)
        cases.append((f"gap_{i}", _ring(rng, th, 1.0 - 1e-6), eps, 5))
    # clusters straddling the +-pi seam
    th = np.concatenate([rng.uniform(3.0, math.pi, 400), rng.uniform(-math.pi, -3.0, 400)])
    cases.append(("seam", _ring(rng, th), 0.2, 8))
    # features off the unit ring (short displacements, arbitrary points)
    z = _ring(rng, rng.normal(1.0, 0.5, 1500))
    z[:60] = rng.normal(0, 0.3, (60, 2)).astype(np.float32)
    z[60:120] *= np.float32(0.5)
    cases.append(("off_ring", z, 0.25, 10))
    # one feature just inside the ring tolerance among 8,191 on it (the
    # terminal point nearest the reference point)
    z = _ring(rng, rng.uniform(-math.pi, math.pi, 8192))
    z[4321] *= np.float32(0.9984)
    cases.append(("one_off_8192", z, 0.25, 20))
    # a sparse stretch between two dense arcs: the block of sorted points
    # that spans it needs more boundary points than its LDS holds
    th = np.concatenate([rng.uniform(0.0, 0.4, 7000), rng.uniform(0.4, 3.0, 600),
                         rng.uniform(3.0, 3.4, 7000)])
    cases.append(("sparse_between_dense", _ring(rng, th), 0.25, 20))
    # one bucket with more points than the bucket-major tables hold (the
    # count pass then scans the keys)
    th = np.concatenate([np.full(300, 1.2345), rng.normal(1.0, 0.4, 2700)])
    cases.append(("crowded_bucket", _ring(rng, th), 0.25, 20))
    # more than 64 clusters
    ang = np.repeat(np.arange(90) * (2 * math.pi / 90), 20) + rng.normal(0, 0.002, 1800)
    cases.append(("90_groups", _ring(rng, ang), 0.03, 5))
    cases.append(("large_eps", _ring(rng, rng.normal(0, 0.6, 2000)), 1.2, 30))
    cases.append(("small_eps", _ring(rng, rng.normal(0, 0.05, 2000)), 0.02, 5))
    cases.append(("duplicates", _ring(rng, np.repeat(rng.uniform(-3, 3, 40), 25), 1.0, 1.0), 0.1, 10))
    cases.append(("two_points", _ring(rng, np.array([0.1, 0.1 + crit])), eps, 1))
    # planners beyond the bitmap's limit (window against the distance passes)
    cases.append(("arc_32768", _ring(rng, rng.normal(-2.0, 0.4, 32768)), 0.25, 20))
    th = np.concatenate([rng.normal(1.0, 0.3, 40000), rng.normal(2.6, 0.2, 25000),
                         rng.uniform(-math.pi, math.pi, 536)])
    z = _ring(rng, th)
    z[:300] = rng.normal(0, 0.4, (300, 2)).astype(np.float32)
    cases.append(("two_arcs_65536", z, 0.25, 20))
    return cases


CASES = _cases()


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_window_matches_bitmap_tiled_and_definition(case):
    from paper_2607_06499_amd import binding as B

    name, z, eps, min_pts = CASES[case]
    V = len(z)
    spec = W.PlannerSpec(num_samples=max(V, 64), horizon=8 if V > 16384 else 50, dbscan_eps=eps,
                         dbscan_min_pts=min_pts).rounded()
    pl = B.Planner(spec)
    assert pl.dbscan_path() == B.DBSCAN_WINDOW
    modes = (B.DBSCAN_WINDOW, B.DBSCAN_TILED) + ((B.DBSCAN_BITMAP,) if V <= 16384 else ())
    res = {}
    for mode in modes:
        pl.set_dbscan_mode(mode)
        lab, cnt, M = pl.stage_dbscan(H.to_dev(z))
        res[mode] = (lab.cpu().numpy(), cnt.cpu().numpy(), int(M.cpu().item()))
        if mode == B.DBSCAN_WINDOW:
            runs = int(pl.debug(B.DBG_TREES, 2).cpu().numpy()[0])
    pl.close()
    lw, cw, mw = res[B.DBSCAN_WINDOW]
    lt, ct, mt = res[B.DBSCAN_TILED]
    print(f"{name}: V={V} M={mw} runs={runs}")
    if B.DBSCAN_BITMAP in res:
        lb, cb, mb = res[B.DBSCAN_BITMAP]
        assert np.array_equal(cw, cb) and np.array_equal(lw, lb) and mw == mb, name
    assert np.array_equal(lw, lt) and mw == mt, name
    assert H.counts_agree(ct, cw, min_pts), name
    eps32 = float(np.float32(eps))
    z64 = z.astype(np.float64)
    if V > 40000:
        # beyond what the brute-force check finishes in seconds: exact FP64
        # counts of sampled points (one row of distances each), every
        # difference explained by a pair within the band of eps
        rng = np.random.default_rng(3)
        lim = 0.5 * H.STAGE_BAND * eps32
        for k in rng.choice(V, 256, replace=False):
            d = np.sqrt(((z64 - z64[k]) ** 2).sum(1))
            exact = int((d <= eps32).sum())
            band = int((np.abs(d - eps32) <= 2 * lim).sum())
            assert abs(int(cw[k]) - exact) <= band, (name, k, cw[k], exact, band)
        return
    olab, _, ocnt, oM = oracle.dbscan(z64, eps32, min_pts)
    if V > 16384 and np.array_equal(cw, ocnt) and np.array_equal(lw, olab):
        print(f"{name}: counts and labels equal to the oracle's")
        return
    st = H.dbscan_check(z64, eps32, min_pts, cw, lw, 0.5 * H.STAGE_BAND * eps32, exact_ref=olab, tag=name)
    print(f"{name}: {st}")
    if st["flagged_pairs"] == 0:
        assert np.array_equal(cw, ocnt) and mw == oM, name


@pytest.mark.parametrize("V", [1, 3, 511, 512, 513, 1023, 1024, 1025, 2047])
def test_window_block_edges(V):
    """Feature counts around the count blocks' 512 positions (one block,
    a block plus one point, exact multiples): window, bitmap and distance
    passes agree bit for bit, and the window result is DBSCAN by the
    definition."""
    from paper_2607_06499_amd import binding as B

    rng = np.random.default_rng(100 + V)
    th = np.concatenate([rng.normal(0.3, 0.2, V - V // 5), rng.uniform(-math.pi, math.pi, V // 5)])
    z = _ring(rng, th)
    if V > 3:
        z[-2:] = rng.normal(0, 0.3, (2, 2)).astype(np.float32)  # two off the ring, sorted last
    eps, min_pts = 0.25, 6
    spec = W.PlannerSpec(num_samples=max(V, 64), dbscan_eps=eps, dbscan_min_pts=min_pts).rounded()
    pl = B.Planner(spec)
    res = {}
    for mode in (B.DBSCAN_WINDOW, B.DBSCAN_BITMAP, B.DBSCAN_TILED):
        pl.set_dbscan_mode(mode)
        lab, cnt, M = pl.stage_dbscan(H.to_dev(z))
        res[mode] = (lab.cpu().numpy(), cnt.cpu().numpy(), int(M.cpu().item()))
    pl.close()
    lw, cw, mw = res[B.DBSCAN_WINDOW]
    lb, cb, mb = res[B.DBSCAN_BITMAP]
    lt, ct, mt = res[B.DBSCAN_TILED]
    assert np.array_equal(cw, cb) and np.array_equal(lw, lb) and np.array_equal(lw, lt) and mw == mb == mt
    assert H.counts_agree(ct, cw, min_pts)
    eps32 = float(np.float32(eps))
    olab = oracle.dbscan(z.astype(np.float64), eps32, min_pts)[0]
    H.dbscan_check(z.astype(np.float64), eps32, min_pts, cw, lw, 0.5 * H.STAGE_BAND * eps32, exact_ref=olab,
                   tag=f"V={V}")


def test_window_repeated_calls_and_all_off_ring():
    """Forty stage calls in a row of random sizes on one planner (the
    bucket tables and the completion ticket start from zero at every call),
    including sets with every point off the ring, each equal to the bitmap's
    result on the same features."""
    from paper_2607_06499_amd import binding as B

    rng = np.random.default_rng(77)
    spec = W.PlannerSpec(num_samples=4096, dbscan_eps=0.2, dbscan_min_pts=8).rounded()
    pw, pb = B.Planner(spec), B.Planner(spec)
    pb.set_dbscan_mode(B.DBSCAN_BITMAP)
    for i in range(40):
        V = int(rng.integers(0, 4097))
        if i % 5 == 4:
            z = (rng.uniform(-0.9, 0.9, (V, 2))).astype(np.float32)  # all off the ring
        else:
            z = _ring(rng, rng.normal(rng.uniform(-3, 3), 0.5, V))
        lw, cw, mw = pw.stage_dbscan(H.to_dev(z))
        lb, cb, mb = pb.stage_dbscan(H.to_dev(z))
        assert np.array_equal(lw.cpu().numpy(), lb.cpu().numpy()), (i, V)
        assert np.array_equal(cw.cpu().numpy(), cb.cpu().numpy()), (i, V)
        assert int(mw.cpu().item()) == int(mb.cpu().item()), (i, V)
    pw.close()
    pb.close()


def _twins(spec):
    from paper_2607_06499_amd import binding as B

    pls = {}
    for mode in (B.DBSCAN_WINDOW, B.DBSCAN_BITMAP, B.DBSCAN_TILED):
        if mode == B.DBSCAN_BITMAP and spec.num_samples > 16384:
            continue
        pl = B.Planner(spec)
        pl.set_dbscan_mode(mode)
        assert pl.dbscan_path() == mode
        pls[mode] = pl
    return pls


REPLANS = [
    ("dynamic_ahead_8192", lambda: W.unicycle_dynamic_ahead(1), 4),
    ("static_ahead_1024", lambda: W.unicycle_static_ahead(2), 4),
    ("crossing_8192", lambda: W.unicycle_crossing(1, side=1, num_samples=8192, distance=1.2), 4),
    ("random_2000", lambda: W.random_scene(11, num_samples=2000, horizon=40, n_obs=10), 3),
    ("paper_unicycle_1", lambda: W.paper_unicycle_preset(1), 4),
    ("dynamic_ahead_32768", lambda: W.unicycle_dynamic_ahead(1, num_samples=32768), 3),
]


@pytest.mark.parametrize("name,make,steps", REPLANS, ids=[r[0] for r in REPLANS])
def test_window_replans_bitwise(name, make, steps):
    """Closed loops with moving obstacles: planners on the three paths replan
    from the same inputs; every output, label, count and cluster statistic
    of the window path equals the bitmap's bit for bit (the tiled counts by
    their contract), step after step."""
    from paper_2607_06499_amd import binding as B

    s = make()
    spec = s.spec
    pls = _twins(spec)
    for pl in pls.values():
        pl.set_nominal(H.to_dev(s.U0))
    fld = s.field.copy()
    x = s.x0.astype(np.float64)
    clustered = 0
    for t in range(steps):
        obs = fld.observation()
        r = {m: H.gpu_replan(pl, np.float32(x), obs) for m, pl in pls.items()}
        w, tl = r[B.DBSCAN_WINDOW], r[B.DBSCAN_TILED]
        bm = r.get(B.DBSCAN_BITMAP, w)
        for k in ("S", "col", "v_idx", "z", "label", "c_mean_cost", "c_dir", "c_size", "u_out", "U_new",
                  "U_next"):
            assert np.array_equal(w[k], bm[k]) and np.array_equal(w[k], tl[k]), (name, t, k)
        assert np.array_equal(w["ncount"], bm["ncount"]), (name, t)
        assert H.counts_agree(tl["ncount"], w["ncount"], spec.dbscan_min_pts), (name, t)
        for k in w["info"]:
            for o in (bm, tl):
                assert np.array_equal(np.asarray(w["info"][k]), np.asarray(o["info"][k])), (name, t, k)
        if w["info"]["branch"] == 0 and w["info"]["n_clusters"] >= 1:
            clustered += 1
        print(f"{name} t={t}: branch={w['info']['branch']} V={len(w['label'])} M={w['info']['n_clusters']}")
        x = unicycle_step(x, w["u_out"], spec.dt)
        fld.step(spec.dt)
    assert clustered >= 1, name


def test_dbscan_mode_availability():
    from paper_2607_06499_amd import binding as B

    arm = B.Planner(W.arm6_dynamic(1, num_samples=512).spec)
    assert arm.dbscan_path() == B.DBSCAN_BITMAP
    with pytest.raises(B.CeMppiError):
        arm.set_dbscan_mode(B.DBSCAN_WINDOW)
    assert arm.dbscan_path() == B.DBSCAN_BITMAP
    big = B.Planner(W.PlannerSpec(num_samples=20000, horizon=8).rounded())
    assert big.dbscan_path() == B.DBSCAN_WINDOW
    with pytest.raises(B.CeMppiError):
        big.set_dbscan_mode(B.DBSCAN_BITMAP)
    assert big.dbscan_path() == B.DBSCAN_WINDOW
    big.set_dbscan_mode(B.DBSCAN_TILED)
    assert big.dbscan_path() == B.DBSCAN_TILED
    tiny_eps = B.Planner(W.PlannerSpec(num_samples=512, dbscan_eps=0.002).rounded())
    assert tiny_eps.dbscan_path() == B.DBSCAN_BITMAP
    pl = B.Planner(W.PlannerSpec(num_samples=512).rounded())
    pl.set_dbscan_mode(B.DBSCAN_TILED)
    assert pl.dbscan_path() == B.DBSCAN_TILED
    pl.set_dbscan_mode(B.DBSCAN_AUTO)
    assert pl.dbscan_path() == B.DBSCAN_WINDOW
    with pytest.raises(B.CeMppiError):
        pl.set_dbscan_mode(7)
    for p in (arm, big, tiny_eps, pl):
        p.close()

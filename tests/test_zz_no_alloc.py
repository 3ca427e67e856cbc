"""The allocation-free DBSCAN entry point (ce_mppi_dbscan_noalloc) against
the planner's stage entry point (ce_mppi_stage_dbscan) that runs the same
kernels out of a planner arena: bitwise equal labels and cluster counts on
two calls in a row, the second with fewer points, in 2-D and 3-D; neighbour
counts equal below minPts (above it a count only has to reach minPts, and
where it stops depends on the order the tiles are visited); both against
the oracle's definition; and the host-side rejection of sizes beyond the
scratch capacity."""
import numpy as np
import pytest

import oracle

from paper_2607_06499_amd import workloads as W
from tests import harness as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not H.gpu_ok():
        pytest.skip("no GPU")


def _features(rng, V, p):
    if p == 2:
        th = np.concatenate([rng.normal(0.6, 0.3, V // 2), rng.normal(-1.4, 0.25, V - V // 2)])
        z = np.stack([np.cos(th), np.sin(th)], 1)
    else:
        v = rng.normal(size=(V, 3))
        v[: V // 2] += 2.5 * np.array([1.0, 0.0, 0.0])
        z = v / np.linalg.norm(v, axis=1, keepdims=True)
    return z.astype(np.float32)


@pytest.mark.parametrize("p,sizes,eps,min_pts", [(2, (9000, 3100), 0.25, 20), (3, (5000, 777), 0.35, 16),
                                                 (2, (16384, 1), 0.2, 12)])
def test_noalloc_matches_stage_dbscan(p, sizes, eps, min_pts):
    from paper_2607_06499_amd import binding as B

    torch = H.torch_mod()
    rng = np.random.default_rng(100 + p)
    spec = W.PlannerSpec(dynamics=W.UNICYCLE if p == 2 else W.ARM6, num_samples=max(sizes),
                         dbscan_eps=eps, dbscan_min_pts=min_pts, dh=W.arm_dh([0.2] * 6)).rounded()
    pl = B.Planner(spec)
    for V in sizes:
        z = H.to_dev(_features(rng, V, p))
        lab_a, cnt_a, M_a = B.dbscan_noalloc(z, spec.dbscan_eps, min_pts)
        torch.cuda.synchronize()
        lab_b, cnt_b, M_b = pl.stage_dbscan(z)
        torch.cuda.synchronize()
        print(f"p={p} V={V}: M={int(M_a.item())}")
        assert torch.equal(lab_a, lab_b), (p, V)
        ca, cb = cnt_a.cpu().numpy(), cnt_b.cpu().numpy()
        low = ca < min_pts
        assert np.array_equal(ca[low], cb[low]) and np.all(cb[~low] >= min_pts), (p, V)
        assert int(M_a.item()) == int(M_b.item()), (p, V)
        zf = z.cpu().numpy().astype(np.float64)
        ol, _, on, oM = oracle.dbscan(zf, float(np.float32(eps)), min_pts)
        st = H.dbscan_check(zf, float(np.float32(eps)), min_pts, ca, lab_a.cpu().numpy(),
                            0.5 * H.STAGE_BAND * float(np.float32(eps)), exact_ref=ol, tag=f"p={p} V={V}")
        print(f"p={p} V={V}: {st}")
    pl.close()


def test_noalloc_rejects_oversize_and_bad_arguments():
    from paper_2607_06499_amd import binding as B

    z = H.to_dev(np.zeros((B.NOALLOC_MAX_POINTS + 1, 2), np.float32))
    with pytest.raises(B.CeMppiError) as e:
        B.dbscan_noalloc(z, 0.3, 5)
    assert e.value.status == B.CE_EINVAL
    z = H.to_dev(np.zeros((10, 4), np.float32))
    with pytest.raises(B.CeMppiError):
        B.dbscan_noalloc(z, 0.3, 5)
    z = H.to_dev(np.zeros((10, 2), np.float32))
    with pytest.raises(B.CeMppiError):
        B.dbscan_noalloc(z, 0.0, 5)
    lab, cnt, M = B.dbscan_noalloc(H.to_dev(np.zeros((0, 2), np.float32)), 0.3, 5)
    assert int(M.item()) == 0 and lab.numel() == 0

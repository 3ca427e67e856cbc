"""Pins of the oracle's DBSCAN (Sec. II-B.2 with the conventions: closed
eps-ball, minPts counts the point itself, border -> lowest-index core
neighbour, clusters numbered by their lowest core index): brute-force
transitive closure on tiny inputs and scikit-learn on larger ones."""
import itertools

import numpy as np
import pytest


def brute_force(pts, eps, min_pts):
    n = len(pts)
    A = np.array([[np.linalg.norm(pts[a] - pts[b]) <= eps for b in range(n)] for a in range(n)])
    core = A.sum(1) >= min_pts
    # transitive closure of the core-core relation (Warshall)
    R = A & core[:, None] & core[None, :]
    for k in range(n):
        R = R | (R[:, k:k + 1] & R[k:k + 1, :])
    lab = -np.ones(n, int)
    M = 0
    for a in range(n):
        if core[a] and lab[a] < 0:
            for b in range(n):
                if R[a, b] or b == a:
                    lab[b] = M
            M += 1
    for a in range(n):
        if not core[a]:
            nb = [b for b in range(n) if core[b] and A[a, b]]
            if nb:
                lab[a] = lab[min(nb)]
    return lab, core, A.sum(1), M


@pytest.mark.parametrize("trial", range(60))
def test_tiny_inputs_against_transitive_closure(orc, trial):
    rng = np.random.default_rng(trial)
    n = int(rng.integers(1, 13))
    # grid points with spacing 0.1: pair distances are 0, 0.1, 0.1414, 0.2, ...,
    # all far from eps = 0.15, so the single-precision decision is unambiguous
    pts = rng.integers(0, 5, size=(n, 2)).astype(float) * 0.1
    if trial % 3 == 0:
        pts[rng.integers(0, n, size=n // 2)] = pts[0]  # duplicates
    for min_pts in (1, 2, 3, 4, 6):
        lab, core, cnt, M = orc.dbscan(pts, 0.15, min_pts)
        blab, bcore, bcnt, bM = brute_force(pts, 0.15, min_pts)
        assert M == bM
        assert np.array_equal(cnt, bcnt)
        assert np.array_equal(core, bcore)
        assert np.array_equal(lab, blab), (pts, min_pts, lab, blab)


def test_chain_at_spacing_just_under_eps(orc):
    # a long chain of points 0.0999 apart with eps 0.1 is one cluster; a gap of
    # 0.1001 splits it
    x = np.concatenate([np.arange(40) * 0.0999, 40 * 0.0999 + 0.1001 + np.arange(10) * 0.0999])
    pts = np.stack([x, np.zeros_like(x)], 1)
    lab, core, cnt, M = orc.dbscan(pts, 0.1, 3)
    assert M == 2
    assert np.all(lab[:40] == 0) and np.all(lab[40:] == 1)
    assert not core[0] and not core[39] and core[1]  # chain ends have 2 neighbours


def _partition(lab, mask):
    groups = {}
    for i in np.nonzero(mask)[0]:
        groups.setdefault(lab[i], []).append(i)
    return sorted(tuple(g) for g in groups.values())


@pytest.mark.parametrize("dim,seed", [(2, 0), (2, 1), (3, 2), (3, 3), (2, 4)])
def test_against_sklearn(orc, dim, seed):
    from sklearn.cluster import DBSCAN

    rng = np.random.default_rng(seed)
    # unit-norm directions in a few lobes, like the clustering feature
    centres = rng.normal(size=(4, dim))
    pts = np.concatenate([c + 0.15 * rng.normal(size=(70, dim)) for c in centres])
    pts /= np.linalg.norm(pts, axis=1, keepdims=True) + 1e-6
    min_pts = 8
    d = np.linalg.norm(pts[:, None] - pts[None], axis=2)
    # the first radius with no pair within 1e-6 of the boundary
    eps = next(e for e in np.arange(0.25, 0.3, 0.001) if np.min(np.abs(d - float(np.float32(e)))) > 1e-6)
    eps = float(np.float32(eps))
    lab, core, cnt, M = orc.dbscan(pts, eps, min_pts)
    sk = DBSCAN(eps=eps, min_samples=min_pts).fit(pts)
    skcore = np.zeros(len(pts), bool)
    skcore[sk.core_sample_indices_] = True
    assert np.array_equal(core, skcore)
    assert np.array_equal(lab < 0, sk.labels_ < 0)
    assert _partition(lab, core) == _partition(sk.labels_, skcore)
    assert M == len(set(sk.labels_) - {-1})
    # canonical numbering: cluster c has the c-th smallest lowest core index
    firsts = [np.min(np.nonzero(core & (lab == c))[0]) for c in range(M)]
    assert firsts == sorted(firsts)


def test_core_partition_invariant_under_permutation(orc):
    rng = np.random.default_rng(11)
    pts = rng.normal(size=(150, 2))
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    lab, core, _, M = orc.dbscan(pts, 0.2, 5)
    perm = rng.permutation(len(pts))
    lab2, core2, _, M2 = orc.dbscan(pts[perm], 0.2, 5)
    assert M == M2
    assert np.array_equal(core[perm], core2)
    inv = np.argsort(perm)
    assert _partition(lab, core) == _partition(lab2[inv], core2[inv])


def test_closed_ball_at_exact_radius(orc):
    # two points exactly eps apart (in single precision) are neighbours
    eps = float(np.float32(0.3))
    pts = np.array([[0.0, 0.0], [eps, 0.0], [5.0, 5.0]])
    lab, core, cnt, M = orc.dbscan(pts, eps, 2)
    assert list(cnt) == [2, 2, 1] and M == 1 and list(lab) == [0, 0, -1]


def test_empty_and_degenerate(orc):
    lab, core, cnt, M = orc.dbscan(np.zeros((0, 2)), 0.3, 2)
    assert M == 0 and lab.size == 0
    pts = np.zeros((5, 2))
    lab, core, cnt, M = orc.dbscan(pts, 0.3, 5)
    assert M == 1 and np.all(lab == 0) and np.all(cnt == 5)
    lab, core, cnt, M = orc.dbscan(pts, 0.3, 6)
    assert M == 0 and np.all(lab == -1)


def test_neighbourhood_decided_in_double_precision(orc):
    # eps promoted from single precision; a pair at exactly eps is inside, a
    # pair 1e-12 farther is outside (single precision could not separate them)
    eps = float(np.float32(0.25))
    pts = np.array([[0.0, 0.0], [eps, 0.0], [0.0, 3.0], [eps + 1e-12, 3.0]])
    lab, core, cnt, M = orc.dbscan(pts, eps, 2)
    assert list(cnt) == [2, 2, 1, 1]
    assert list(lab) == [0, 0, -1, -1] and M == 1
    # the same in three dimensions, along a diagonal: |d|^2 = 3 (eps/sqrt3)^2
    d = eps / np.sqrt(3.0)
    p3 = np.array([[0.0, 0.0, 0.0], [d, d, d], [5.0, 5.0, 5.0], [5.0 + d * (1 + 1e-9), 5.0 + d, 5.0 + d]])
    _, _, cnt3, _ = orc.dbscan(p3, eps, 2)
    inside = 3 * d * d <= eps * eps
    assert list(cnt3[:2]) == ([2, 2] if inside else [1, 1])
    assert list(cnt3[2:]) == [1, 1]

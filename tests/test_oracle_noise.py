"""Pins of the oracle's noise generator (Sec. II-A: eps ~ N(0, Sigma)).

Philox4x32-10 is checked word for word against an independent
implementation (PyTorch's header-only engine), the uniforms against their
exact closed form, and the Gaussians statistically."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2607_06499_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def _torch_include():
    try:
        import torch
    except Exception:  # pragma: no cover
        return None
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    return inc if os.path.exists(os.path.join(inc, "ATen/core/PhiloxRNGEngine.h")) else None


@pytest.fixture(scope="module")
def philox_ref():
    inc = _torch_include()
    if inc is None or shutil.which("g++") is None:
        pytest.skip("PyTorch headers or g++ not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "philox_ref")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", inc,
                    os.path.join(HERE, "helpers", "philox_torch_ref.cpp"), "-o", exe], check=True)
    yield exe
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_independent_engine(orc, philox_ref):
    rng = np.random.default_rng(7)
    cases = [np.zeros(6, np.uint64), np.full(6, 0xFFFFFFFF, np.uint64)]
    cases += [rng.integers(0, 2**32, size=6, dtype=np.uint64) for _ in range(300)]
    # the layouts the planner uses: (block, rollout, step, stream) / (seed lo, seed hi)
    cases += [np.array([b, k, 17, 3, 12345, 0], np.uint64) for b in range(4) for k in range(0, 9000, 997)]
    text = "\n".join(" ".join(str(int(v)) for v in c) for c in cases) + "\n"
    out = subprocess.run([philox_ref], input=text, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], np.uint64)
    for c, r in zip(cases, ref):
        got = orc.philox4x32_10(c[:4].astype(np.uint32), c[4:].astype(np.uint32))
        assert np.array_equal(got.astype(np.uint64), r), (c, got, r)


def test_uniform_closed_form(orc):
    # (2*(w>>9)+1) * 2^-24: endpoints and exact single-precision values
    assert orc.uniform(0) == 2.0**-24
    assert orc.uniform(0xFFFFFFFF) == 1.0 - 2.0**-24
    rng = np.random.default_rng(3)
    for w in rng.integers(0, 2**32, size=2000):
        u = orc.uniform(int(w))
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
        assert u == ((int(w) >> 9) * 2 + 1) / 2.0**24


def test_box_muller_radius_and_angle(orc):
    # r^2 = -2 ln u_a and atan2(g_b, g_a) = 2 pi u_b (mod 2 pi)
    rng = np.random.default_rng(4)
    for wa, wb in rng.integers(0, 2**32, size=(500, 2)):
        ga, gb = orc.box_muller(int(wa), int(wb))
        ua, ub = orc.uniform(int(wa)), orc.uniform(int(wb))
        assert ga * ga + gb * gb == pytest.approx(-2.0 * np.log(ua), rel=1e-12, abs=1e-15)
        ang = np.arctan2(gb, ga) % (2 * np.pi)
        d = abs(ang - 2 * np.pi * ub)
        assert min(d, 2 * np.pi - d) < 1e-9


def _spec(L, m_dyn=W.UNICYCLE, N=40, seed=5, stream=2):
    s = W.PlannerSpec(dynamics=m_dyn, horizon=N, num_samples=1, noise_chol=L, seed=seed,
                      stream_id=stream)
    return s.rounded()


def test_gaussians_statistics(orc):
    from scipy import stats

    spec = _spec(W.diag_chol([1.0, 1.0], 2))
    g = np.concatenate([orc.rollout_noise(spec, 11, k)[0].ravel() for k in range(2500)])
    assert g.size == 2500 * 80
    assert abs(g.mean()) < 5.0 / np.sqrt(g.size)
    assert abs(g.var() - 1.0) < 5.0 * np.sqrt(2.0 / g.size)
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # the two members of a Box-Muller pair and neighbouring pairs are uncorrelated
    pairs = g.reshape(-1, 2)
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 5.0 / np.sqrt(pairs.shape[0])
    quads = g.reshape(-1, 4)
    assert abs(np.corrcoef(quads[:, 0], quads[:, 2])[0, 1]) < 5.0 / np.sqrt(quads.shape[0])


def test_noise_covariance_is_LLt(orc):
    # eps = L g has covariance Sigma = L L^T (full lower-triangular L, arm)
    L = np.array([[0.3, 0, 0, 0, 0, 0], [0.1, 0.2, 0, 0, 0, 0], [-0.05, 0.1, 0.4, 0, 0, 0],
                  [0, 0, 0.2, 0.1, 0, 0], [0.2, 0, 0, 0, 0.3, 0], [0, -0.1, 0, 0.1, 0, 0.25]])
    spec = _spec(list(L.ravel()), W.ARM6, N=20)
    L32 = np.asarray(spec.noise_chol, np.float64).reshape(6, 6)
    eps = np.concatenate([orc.rollout_noise(spec, 0, k)[1] for k in range(3000)])
    Sigma = L32 @ L32.T
    C = np.cov(eps.T)
    assert np.max(np.abs(C - Sigma)) < 6.0 * 0.45**2 / np.sqrt(eps.shape[0]) * 2


def test_noise_depends_on_every_counter_word(orc):
    base = _spec(W.diag_chol([1.0, 1.0], 2), seed=9, stream=1)
    w = orc.noise_words(base, 5, 3)
    assert not np.array_equal(w, orc.noise_words(base, 6, 3))           # step
    assert not np.array_equal(w, orc.noise_words(base, 5, 4))           # rollout
    assert not np.array_equal(w, orc.noise_words(base.replace(stream_id=2), 5, 3))
    assert not np.array_equal(w, orc.noise_words(base.replace(seed=9 + (1 << 32)), 5, 3))
    # block b of rollout k is Philox((b, k, step, stream), (seed lo, seed hi))
    for b in range(len(w) // 4):
        ref = orc.philox4x32_10([b, 3, 5, 1], [9, 0])
        assert np.array_equal(w[4 * b:4 * b + 4], ref)


def test_noise_element_layout(orc):
    # element e = j*m+i of rollout k is member (e mod 2) of the Box-Muller pair
    # fed by words (0,1) or (2,3) of block e//4
    spec = _spec(W.diag_chol([1.0, 1.0], 2), N=7)
    w = orc.noise_words(spec, 2, 8)
    g, eps = orc.rollout_noise(spec, 2, 8)
    flat = g.ravel()
    for e in range(flat.size):
        b, h = e // 4, (e // 2) % 2
        ga, gb = orc.box_muller(int(w[4 * b + 2 * h]), int(w[4 * b + 2 * h + 1]))
        assert flat[e] == (ga if e % 2 == 0 else gb)
    assert np.array_equal(eps, g)  # identity L

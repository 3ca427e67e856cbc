"""Pins of the path-integral update (Eq. (6)-(7), Eq. (19)-(20))."""
import numpy as np
import pytest


def _data(K=40, N=6, m=2, seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(size=K) * 3 + 10, rng.normal(size=(K, N, m)), rng.normal(size=(N, m))


def test_weights_sum_to_one_and_match_softmax_ratios(orc):
    S, E, U = _data()
    idx = np.arange(0, 40, 3)
    Un, w, smin = orc.weighted_update(idx, S, E, 0.7, U)
    assert w[idx].sum() == pytest.approx(1.0, abs=1e-14)
    assert np.all(w[np.setdiff1d(np.arange(40), idx)] == 0)
    assert smin == S[idx].min()
    # ratios follow exp(-(S_a - S_b)/lambda)
    a, b = idx[0], idx[1]
    assert w[a] / w[b] == pytest.approx(np.exp(-(S[a] - S[b]) / 0.7), rel=1e-12)
    assert np.allclose(Un, U + np.tensordot(w, E, axes=(0, 0)), atol=1e-13)


def test_constant_cost_is_plain_mean(orc):
    _, E, U = _data(seed=1)
    S = np.full(40, 123.0)
    idx = np.arange(5, 30)
    Un, w, _ = orc.weighted_update(idx, S, E, 0.3, U)
    assert np.allclose(Un, U + E[idx].mean(0), atol=1e-13)


def test_temperature_limits(orc):
    S, E, U = _data(seed=2)
    idx = np.arange(40)
    Un, _, _ = orc.weighted_update(idx, S, E, 1e12, U)
    assert np.allclose(Un, U + E.mean(0), atol=1e-9)
    Un, _, _ = orc.weighted_update(idx, S, E, 1e-6, U)
    assert np.allclose(Un, U + E[np.argmin(S)], atol=1e-12)


def test_shift_invariance_in_cost(orc):
    S, E, U = _data(seed=3)
    idx = np.arange(0, 40, 2)
    a, _, _ = orc.weighted_update(idx, S, E, 0.5, U)
    b, _, _ = orc.weighted_update(idx, S + 1e4, E, 0.5, U)
    assert np.allclose(a, b, atol=1e-12)


def test_single_member(orc):
    S, E, U = _data(seed=4)
    Un, w, _ = orc.weighted_update([7], S, E, 0.5, U)
    assert np.allclose(Un, U + E[7], atol=0)

"""Pins of the oracle's discounted returns and GAE (FP64)."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle as O

# G_0 = (1 - gamma^T) / (1 - gamma) for r = 1, no dones, no bootstrap, gamma = 0.99
CLOSED = {8: 7.725530557208, 200: 86.602032514204, 250: 91.894148383782,
          500: 99.342951695758, 1000: 99.995682875259}


@pytest.mark.parametrize("T", sorted(CLOSED))
def test_constant_reward_geometric_series(T):
    rows = 3
    r = np.ones((T, rows))
    v = np.zeros((T, rows))
    d = np.zeros((T, rows), np.uint8)
    ret, adv = O.returns_gae(r, v, d, np.zeros(rows), 0.99, 0.95, bootstrap=False)
    assert ret[0, 0] == pytest.approx((1 - 0.99**T) / (1 - 0.99), rel=1e-13)
    assert ret[0, 0] == pytest.approx(CLOSED[T], abs=1e-11)
    # every later index is the same series with a shorter horizon
    k = T // 2
    assert ret[k, 1] == pytest.approx((1 - 0.99 ** (T - k)) / (1 - 0.99), rel=1e-13)


@settings(max_examples=120, deadline=None)
@given(T=st.integers(1, 8), rows=st.integers(1, 4), seed=st.integers(0, 2**31 - 1),
       gamma=st.floats(0.0, 1.0), lam=st.floats(0.0, 1.0), boot=st.booleans(),
       p_done=st.sampled_from([0.0, 0.3, 1.0]))
def test_recursion_equals_bruteforce_sums(T, rows, seed, gamma, lam, boot, p_done):
    rng = np.random.default_rng(seed)
    r = rng.normal(size=(T, rows))
    v = rng.normal(size=(T, rows))
    d = (rng.random((T, rows)) < p_done).astype(np.uint8)
    lv = rng.normal(size=rows)
    g1, a1 = O.returns_gae(r, v, d, lv, gamma, lam, boot)
    g2, a2 = O.gae_bruteforce(r, v, d, lv, gamma, lam, boot)
    assert np.allclose(g1, g2, rtol=1e-12, atol=1e-12)
    assert np.allclose(a1, a2, rtol=1e-12, atol=1e-12)


def _rand(T=50, rows=6, seed=0, p=0.1):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(T, rows)), rng.normal(size=(T, rows)),
            (rng.random((T, rows)) < p).astype(np.uint8), rng.normal(size=rows))


def test_lambda_one_gives_return_minus_value():
    r, v, d, lv = _rand()
    g, a = O.returns_gae(r, v, d, lv, 0.97, 1.0, True)
    assert np.allclose(a, g - v, atol=1e-12)


def test_lambda_zero_gives_td_error():
    r, v, d, lv = _rand(seed=1)
    g, a = O.returns_gae(r, v, d, lv, 0.97, 0.0, True)
    v_next = np.vstack([v[1:], lv[None]])
    assert np.allclose(a, r + 0.97 * (1 - d) * v_next - v, atol=1e-14)


def test_gamma_zero_is_myopic():
    r, v, d, lv = _rand(seed=2)
    g, a = O.returns_gae(r, v, d, lv, 0.0, 0.95, True)
    assert np.array_equal(g, r) and np.allclose(a, r - v, atol=1e-15)


def test_done_splits_into_independent_segments():
    """A done at t cuts the sequence: the head equals a roll-out that ends
    at t without bootstrap, the tail is unaffected by the head."""
    T, rows = 40, 4
    r, v, d, lv = _rand(T, rows, seed=3, p=0.0)
    cut = 17
    d[cut] = 1
    g, a = O.returns_gae(r, v, d, lv, 0.99, 0.9, True)
    gh, ah = O.returns_gae(r[:cut + 1], v[:cut + 1], d[:cut + 1], np.zeros(rows), 0.99, 0.9, False)
    gt, at = O.returns_gae(r[cut + 1:], v[cut + 1:], d[cut + 1:], lv, 0.99, 0.9, True)
    assert np.allclose(g[:cut + 1], gh, atol=1e-13) and np.allclose(a[:cut + 1], ah, atol=1e-13)
    assert np.allclose(g[cut + 1:], gt, atol=1e-13) and np.allclose(a[cut + 1:], at, atol=1e-13)


def test_bootstrap_adds_discounted_tail_value():
    r, v, d, lv = _rand(T=30, rows=5, seed=4, p=0.0)
    g1, _ = O.returns_gae(r, v, d, lv, 0.95, 0.9, True)
    g0, _ = O.returns_gae(r, v, d, lv, 0.95, 0.9, False)
    T = r.shape[0]
    for t in (0, 10, T - 1):
        assert np.allclose(g1[t] - g0[t], 0.95 ** (T - t) * lv, atol=1e-13)

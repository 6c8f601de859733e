"""Pins of the oracle's policy MLP and action sampling."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F
from scipy import special, stats

import oracle as O
from paper_2408_00930_amd import inputs


def _torch_forward(pol, obs, quant):
    """The policy by torch.nn.functional in float64, with the quantisation
    points applied by torch's own casts (library reference)."""
    x = torch.from_numpy(np.atleast_2d(obs).astype(np.float64))
    Ws = [torch.from_numpy(pol.exact(n)) for n in ("w1", "w2", "w3")]
    bs = [torch.from_numpy(pol.exact(n)) for n in ("b1", "b2", "b3")]
    for i in range(3):
        x = quant(x)
        x = F.linear(x, Ws[i], bs[i])
        if i < 2:
            x = torch.tanh(x)
    return x.numpy()


def _q_bf16(x):
    return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _q_fp8(scales):
    it = iter(scales)

    def q(x):
        s = next(it)
        return (x / s).to(torch.float32).to(torch.float8_e4m3fn).to(torch.float64) * s
    return q


def test_mlp_f32_matches_torch_linear_chain():
    pol = inputs.make_policy(5, 7, 3, 4, "f32", seed=1)   # non-square: catches transposes
    obs = np.random.default_rng(0).normal(size=(20, 5))
    got = O.mlp_forward(pol, obs)
    want = _torch_forward(pol, obs, lambda x: x)
    assert got.shape == (20, 5)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-14)


def test_mlp_bf16_quantisation_points():
    pol = inputs.make_policy(6, 16, 24, 1, "bf16", seed=2)
    obs = np.random.default_rng(1).normal(size=(30, 6))
    # inputs rounded from float32 values so torch's f32 -> bf16 cast is exact RNE
    obs = obs.astype(np.float32).astype(np.float64)
    got = O.mlp_forward(pol, obs)
    want = _torch_forward(pol, obs, _q_bf16)
    # tanh outputs are rounded from float64 (oracle) vs via float32 (torch):
    # they can differ only where that double rounding moves a tie
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_mlp_fp8_quantisation_points():
    pol = inputs.make_policy(20, 32, 32, 4, "fp8", seed=3)
    obs = np.random.default_rng(2).uniform(-3, 3, size=(30, 20))
    obs = obs.astype(np.float32).astype(np.float64)
    got = O.mlp_forward(pol, obs)
    assert pol.act_scale == (2.0 ** -4, 2.0 ** -8, 2.0 ** -8)
    want = _torch_forward(pol, obs, _q_fp8(pol.act_scale))
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def test_mlp_zero_weights_give_biases():
    pol = inputs.make_policy(4, 8, 8, 2, "f32", seed=4)
    for n in ("w1", "w2", "w3"):
        getattr(pol, n)[:] = 0
    out = O.mlp_forward(pol, np.ones((3, 4)))
    assert np.array_equal(out, np.tile(pol.exact("b3"), (3, 1)))


def test_mlp_structured_weights():
    """W1 selects inputs, W2 is the identity, W3 picks single units: the
    outputs are tanh(tanh(x_i + b1) + b2) + b3 for the selected units."""
    pol = inputs.make_policy(3, 5, 5, 2, "f32", seed=5)
    pol.w1[:] = 0
    pol.w1[0, 2] = pol.w1[1, 0] = pol.w1[2, 1] = pol.w1[3, 2] = pol.w1[4, 0] = 1.0
    pol.w2[:] = np.eye(5, dtype=np.float32)
    pol.w3[:] = 0
    pol.w3[0, 1] = 1.0   # unit 1 <- x0
    pol.w3[1, 3] = 2.0   # unit 3 <- x2
    pol.w3[2, 4] = -1.0  # value: unit 4 <- x0
    x = np.array([0.3, -0.7, 1.1])
    b1, b2, b3 = pol.exact("b1"), pol.exact("b2"), pol.exact("b3")
    unit = lambda j, xi: np.tanh(np.tanh(xi + b1[j]) + b2[j])  # noqa: E731
    out = O.mlp_forward(pol, x)[0]
    assert out[0] == pytest.approx(unit(1, x[0]) + b3[0], abs=1e-15)
    assert out[1] == pytest.approx(2 * unit(3, x[2]) + b3[1], abs=1e-15)
    assert out[2] == pytest.approx(-unit(4, x[0]) + b3[2], abs=1e-15)


# ------------------------------------------------------------ sampling ----

def test_categorical_two_actions_logistic():
    rng = np.random.default_rng(0)
    for _ in range(500):
        l = rng.normal(0, 3, 2)
        u = (2 * rng.integers(0, 2**23) + 1) * 2.0**-24
        a, lp, mg = O.sample_categorical(l, u)
        p0 = special.expit(l[0] - l[1])              # logistic function
        assert a == (0 if u < p0 else 1)
        want = -np.logaddexp(0, l[1] - l[0]) if a == 0 else -np.logaddexp(0, l[0] - l[1])
        assert lp == pytest.approx(want, abs=1e-13)
        assert mg == pytest.approx(abs(u - p0), abs=1e-15)


def test_categorical_equal_logits_is_floor():
    rng = np.random.default_rng(1)
    for K in (2, 3, 40, 50):
        for _ in range(300):
            u = (2 * rng.integers(0, 2**23) + 1) * 2.0**-24
            a, lp, mg = O.sample_categorical(np.full(K, 0.7), u)
            if mg > 1e-12:
                assert a == int(np.floor(u * K))
            assert lp == pytest.approx(-np.log(K), abs=1e-13)


def test_categorical_margin_and_logp_library():
    rng = np.random.default_rng(2)
    for _ in range(300):
        l = rng.normal(0, 2, 50)
        u = rng.uniform()
        a, lp, mg = O.sample_categorical(l, u)
        cdf = np.cumsum(special.softmax(l))
        assert a == int(np.searchsorted(cdf, u, side="right")) or mg < 1e-12
        assert lp == pytest.approx(special.log_softmax(l)[a], abs=1e-12)
        assert mg == pytest.approx(np.min(np.abs(u - cdf[:-1])), abs=1e-12)


def test_categorical_frequencies_chi2():
    rng = np.random.default_rng(3)
    l = rng.normal(0, 1, 10)
    n = 20000
    counts = np.zeros(10)
    for u in rng.uniform(size=n):
        counts[O.sample_categorical(l, u)[0]] += 1
    assert stats.chisquare(counts, special.softmax(l) * n).pvalue > 1e-4


def test_gaussian_logpdf_library():
    rng = np.random.default_rng(4)
    for _ in range(200):
        d = int(rng.integers(1, 3))
        mu, ls, z = rng.normal(size=d), rng.normal(-0.5, 0.3, d), rng.normal(size=d)
        a, lp = O.sample_gaussian(mu, ls, z)
        assert np.allclose(a, mu + np.exp(ls) * z, rtol=1e-15)
        want = stats.norm.logpdf(a, loc=mu, scale=np.exp(ls)).sum()
        assert lp == pytest.approx(want, abs=1e-11)


def test_gaussian_zero_noise_returns_mean():
    a, lp = O.sample_gaussian([0.25], [-0.5], [0.0])
    assert a[0] == 0.25
    assert lp == pytest.approx(0.5 - 0.5 * np.log(2 * np.pi), abs=1e-15)


def test_sample_rows_is_the_per_row_draw_and_sample():
    """The batched draw equals the per-row composition of the pinned parts."""
    rng = np.random.default_rng(12)
    head = rng.normal(size=(30, 6))
    rows = rng.integers(0, 2 ** 31, 30)
    a, lp, mg = O.sample_rows(head, 5, None, 9, 17, rows, 3)
    for i, r in enumerate(rows):
        w = O.draw(9, 17, int(r), O.ACTION, 0, 3)
        want = O.sample_categorical(head[i, :5], O.u01(w[0]))
        assert (a[i], lp[i], mg[i]) == want
    ls = np.array([-0.5])
    a, lp, mg = O.sample_rows(head[:, :2], 0, ls, 9, 17, rows, 3)
    for i, r in enumerate(rows):
        w = O.draw(9, 17, int(r), O.ACTION, 0, 3)
        z0, _ = O.box_muller(O.u01(w[0]), O.u01(w[1]))
        ga, glp = O.sample_gaussian(head[i, :1], ls, [z0])
        assert a[i] == ga[0] and lp[i] == glp and np.isinf(mg[i])

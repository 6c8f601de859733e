"""Pins of the oracle's actor-critic gradient and Adam step.

The gradient is checked against central finite differences of the loss,
which the test evaluates from its definition with the oracle's forward pass
only (an FP32 policy has no rounding, so the loss is smooth in every weight).
Special cases (zero advantage, value-only and entropy-only losses) have
closed forms; the rounded backward of BF16 policies stays within the
rounding it adds. Adam's first step has a closed form."""
import numpy as np
import pytest

import oracle as O

LOG2PI = np.log(2.0 * np.pi)


def _policy(rng, d_in, h, n_head, dtype="f32"):
    w = [rng.normal(0, 0.4, (h, d_in)), rng.normal(0, 0.1, h), rng.normal(0, 0.2, (h, h)),
         rng.normal(0, 0.1, h), rng.normal(0, 0.3, (n_head, h)), rng.normal(0, 0.1, n_head)]
    if dtype == "bf16":
        w = [O.round_bf16(a) for a in w]
    return w


def _hold(w, dtype="f32"):
    return O._MlpHold(dtype, *w)


def _loss(w, n_act, log_std, obs, act, adv, ret, cv, ce):
    """The loss from its definition, with the oracle's forward pass."""
    head = O.mlp_forward(_hold(w), obs)
    v = head[:, -1]
    if n_act == 0:
        mu = head[:, 0]
        sigma = np.exp(log_std)
        logp = -0.5 * ((act - mu) / sigma) ** 2 - log_std - 0.5 * LOG2PI
        ent = np.full(len(obs), log_std + 0.5 * (1.0 + LOG2PI))
    else:
        lg = head[:, :n_act]
        lse = np.log(np.exp(lg - lg.max(1, keepdims=True)).sum(1)) + lg.max(1)
        logp = lg[np.arange(len(obs)), act.astype(int)] - lse
        p = np.exp(lg - lse[:, None])
        ent = -(p * np.log(p)).sum(1)
    return np.mean(-adv * logp + 0.5 * cv * (v - ret) ** 2 - ce * ent)


def _case(seed, n_act, n=6, d_in=3, h=8):
    rng = np.random.default_rng(seed)
    n_head = (n_act if n_act else 1) + 1
    w = _policy(rng, d_in, h, n_head)
    obs = rng.normal(0, 1, (n, d_in))
    act = rng.integers(0, n_act, n).astype(np.float64) if n_act else rng.normal(0, 1, n)
    adv = rng.normal(0, 1, n)
    ret = rng.normal(0, 1, n)
    return w, obs, act, adv, ret


NAMES = ("w1", "b1", "w2", "b2", "w3", "b3")


@pytest.mark.parametrize("n_act", [0, 3])
def test_ac_grad_matches_finite_differences(n_act):
    w, obs, act, adv, ret = _case(1 + n_act, n_act)
    log_std = -0.3
    cv, ce = 0.7, 0.05
    g = O.ac_grad(_hold(w), n_act, obs, act, adv, ret, cv, ce, quant_backward=False,
                  log_std=np.array([log_std]))
    eps = 1e-6
    for name, arr in zip(NAMES, w):
        fd = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            wp = [a.copy() for a in w]
            wm = [a.copy() for a in w]
            k = NAMES.index(name)
            wp[k][idx] += eps
            wm[k][idx] -= eps
            fd[idx] = (_loss(wp, n_act, log_std, obs, act, adv, ret, cv, ce) -
                       _loss(wm, n_act, log_std, obs, act, adv, ret, cv, ce)) / (2 * eps)
        scale = max(1e-3, np.abs(fd).max())
        assert np.abs(g[name] - fd).max() <= 1e-7 * scale + 1e-10, name
    if n_act == 0:
        fd = (_loss(w, 0, log_std + eps, obs, act, adv, ret, cv, ce) -
              _loss(w, 0, log_std - eps, obs, act, adv, ret, cv, ce)) / (2 * eps)
        assert abs(g["log_std"][0] - fd) <= 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("n_act", [0, 4])
def test_ac_grad_special_cases(n_act):
    w, obs, act, adv, ret = _case(7, n_act, n=9)
    hold = _hold(w)
    zero = O.ac_grad(hold, n_act, obs, act, np.zeros(9), ret, 0.0, 0.0, False,
                     log_std=np.array([0.2]))
    for k, v in zero.items():
        assert not v.any(), k
    # value-only loss: the value bias gradient is c_v * mean(V - G), and only
    # the value row of the head receives gradient
    cv = 1.3
    head = O.mlp_forward(hold, obs)
    vo = O.ac_grad(hold, n_act, obs, act, np.zeros(9), ret, cv, 0.0, False,
                   log_std=np.array([0.2]))
    assert np.isclose(vo["b3"][-1], cv * np.mean(head[:, -1] - ret), rtol=1e-13, atol=1e-15)
    assert not vo["b3"][:-1].any() and not vo["w3"][:-1].any()
    # linearity in the advantages (policy part only)
    a1, a2 = np.random.default_rng(3).normal(0, 1, (2, 9))
    g1 = O.ac_grad(hold, n_act, obs, act, a1, ret, 0.0, 0.0, False, log_std=np.array([0.2]))
    g2 = O.ac_grad(hold, n_act, obs, act, a2, ret, 0.0, 0.0, False, log_std=np.array([0.2]))
    g12 = O.ac_grad(hold, n_act, obs, act, a1 + a2, ret, 0.0, 0.0, False,
                    log_std=np.array([0.2]))
    for k in g12:
        assert np.allclose(g12[k], g1[k] + g2[k], rtol=1e-12, atol=1e-15), k


def test_gaussian_entropy_gradient_is_minus_coefficient():
    w, obs, act, adv, ret = _case(11, 0)
    g = O.ac_grad(_hold(w), 0, obs, act, np.zeros(6), ret, 0.0, 0.25, False,
                  log_std=np.array([-0.5]))
    assert np.isclose(g["log_std"][0], -0.25, rtol=1e-15, atol=0)   # six terms of -c_e / n
    assert not g["w1"].any() and not g["b3"].any()


def test_bf16_rounded_backward_stays_within_its_rounding():
    rng = np.random.default_rng(5)
    w = _policy(rng, 3, 32, 2, "bf16")
    obs = rng.normal(0, 1, (40, 3))
    act, adv, ret = rng.normal(0, 1, 40), rng.normal(0, 1, 40), rng.normal(0, 1, 40)
    hold = _hold(w, "bf16")
    exact = O.ac_grad(hold, 0, obs, act, adv, ret, 0.5, 0.0, False, log_std=np.array([-0.5]))
    rounded = O.ac_grad(hold, 0, obs, act, adv, ret, 0.5, 0.0, True, log_std=np.array([-0.5]))
    # biases and log_std never meet a rounded operand of their own layer
    assert np.array_equal(exact["b3"], rounded["b3"])
    assert np.array_equal(exact["log_std"], rounded["log_std"])
    # each rounding is 2^-9 relative; three of them compound through layer 1
    for k in ("w3", "w2", "b2", "w1", "b1"):
        scale = np.abs(exact[k]).max()
        assert np.abs(rounded[k] - exact[k]).max() <= 4 * 2.0 ** -9 * scale * 8, k


def test_fp8_policy_is_rejected():
    rng = np.random.default_rng(0)
    w = _policy(rng, 3, 8, 2)
    with pytest.raises(ValueError):
        O.ac_grad(_hold(w, "fp8"), 0, rng.normal(0, 1, (2, 3)), np.zeros(2), np.ones(2),
                  np.zeros(2), log_std=np.array([0.0]))


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(9)
    g = rng.normal(0, 1, 50)
    theta = rng.normal(0, 1, 50)
    m, v = np.zeros(50), np.zeros(50)
    t0 = theta.copy()
    O.adam(theta, g, m, v, 1, 1e-3, 0.9, 0.999, 0.0)
    # bias-corrected m and v are g and g^2 at step 1: the step is lr * sign(g)
    assert np.allclose(theta, t0 - 1e-3 * np.sign(g), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g, rtol=1e-15) and np.allclose(v, 0.001 * g * g, rtol=1e-15)
    # a second step from the definition, written out
    g2 = rng.normal(0, 1, 50)
    m_w, v_w = 0.9 * m + 0.1 * g2, 0.999 * v + 0.001 * g2 * g2
    want = theta - 1e-3 * (m_w / (1 - 0.9 ** 2)) / (np.sqrt(v_w / (1 - 0.999 ** 2)) + 1e-8)
    O.adam(theta, g2, m, v, 2, 1e-3, 0.9, 0.999, 1e-8)
    assert np.allclose(theta, want, rtol=1e-14, atol=1e-16)


def test_adam_constant_gradient_steps_by_lr():
    """With a constant gradient the bias-corrected moments are g and g^2 at
    every step, so (eps = 0) each step moves every weight by lr * sign(g)."""
    rng = np.random.default_rng(12)
    g = rng.normal(0, 1, 40)
    theta = rng.normal(0, 1, 40)
    m, v = np.zeros(40), np.zeros(40)
    t0 = theta.copy()
    for t in range(1, 26):
        O.adam(theta, g, m, v, t, 2e-3, 0.8, 0.99, 0.0)
        assert np.allclose(theta, t0 - 2e-3 * t * np.sign(g), rtol=0, atol=1e-12), t

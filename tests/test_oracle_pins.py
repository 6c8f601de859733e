"""Hand-computed pins of oracle parts that the other pins leave open: the
Pendulum cost and its pre-step convention, every kind's reset map from an
explicit Philox block, the market's state entries s0..s3 on a three-agent
environment, the observation encodings at special angles, and the places
where the BF16 backward rounds its operands.

Expected values are literals worked out by hand from the written
specification of each environment (the numbers in the comments), or an
independent computation (torch autograd in FP64 with torch's bf16 casts)."""
import math

import numpy as np
import pytest

import oracle as O


def _env(kind, n=1, offsets=None, params=None):
    return O.env_hold(kind, n, offsets, params)


def _u(word):
    """Uniform of one 32-bit word: (2 * (w >> 9) + 1) * 2^-24."""
    return (2 * (int(word) >> 9) + 1) / 16777216.0


# ------------------------------------------------------------ Pendulum ----

def test_pendulum_cost_at_a_general_state():
    """theta = 3.5 wraps to 3.5 - 2 pi = -2.7831853071795862; the cost is
    wrap^2 + 0.1 thd^2 + 0.001 u^2 = 7.7461204541003275 + 0.4 + 0.00225."""
    env = _env(O.PENDULUM)
    nxt, r, done, _ = O.env_step_row(env, [3.5, 2.0], 1.5)
    assert r == pytest.approx(-8.148370454100327, rel=1e-15)
    # a swap of the rate and torque coefficients would give
    # -(7.7461204541003275 + 0.004 + 0.225)
    assert abs(r + 7.9751204541003275) > 0.1
    assert not done


def test_pendulum_cost_uses_the_pre_step_state_and_clipped_torque():
    env = _env(O.PENDULUM)
    s = [0.5, -3.0]                       # the step moves theta and the rate
    nxt, r, _, _ = O.env_step_row(env, s, 7.0)
    assert abs(nxt[0] - s[0]) > 0.05 and abs(nxt[1] - s[1]) > 0.05
    # 0.25 + 0.1 * 9 + 0.001 * 2^2 (torque clipped to 2)
    assert r == pytest.approx(-(0.25 + 0.9 + 0.004), rel=1e-15)


# --------------------------------------------------------------- resets ----

SEED, EPOCH, T, ROW = 0x0123456789ABCDEF, 6, 41, 9


@pytest.mark.parametrize("kind,lo,width", [(O.CARTPOLE, -0.05, 0.1), (O.ACROBOT, -0.1, 0.2)])
def test_uniform_box_resets_map_one_block(kind, lo, width):
    """state[i] = lo + width * u(w[i]) from the RESET block (t, row, sub 0)."""
    w = O.draw(SEED, T, ROW, O.RESET, 0, EPOCH)
    s = O.reset_row(_env(kind, ROW + 1), SEED, EPOCH, T, ROW)
    want = [lo + width * _u(w[i]) for i in range(4)]
    assert np.array_equal(s, want)


def test_pendulum_reset_maps_one_block():
    """theta = -pi + 2 pi u(w0), rate = -1 + 2 u(w1)."""
    w = O.draw(SEED, T, ROW, O.RESET, 0, EPOCH)
    s = O.reset_row(_env(O.PENDULUM, ROW + 1), SEED, EPOCH, T, ROW)
    assert s[0] == -math.pi + 2.0 * math.pi * _u(w[0])
    assert s[1] == -1.0 + 2.0 * _u(w[1])


def test_market_reset_is_box_muller_over_eight_blocks():
    """Entries 4 sub .. 4 sub + 3 come from RESET sub-block `sub`: the cos and
    sin normals of (w0, w1), then of (w2, w3)."""
    offsets = np.array([0, 3, ROW + 5], np.int32)
    s = O.reset_row(_env(O.MARKET, 2, offsets), SEED, EPOCH, T, ROW)
    for sub in range(8):
        w = O.draw(SEED, T, ROW, O.RESET, sub, EPOCH)
        for pair in range(2):
            u1, u2 = _u(w[2 * pair]), _u(w[2 * pair + 1])
            rad = math.sqrt(-2.0 * math.log(u1))
            assert s[4 * sub + 2 * pair] == pytest.approx(rad * math.cos(2 * math.pi * u2),
                                                          rel=1e-14, abs=1e-15)
            assert s[4 * sub + 2 * pair + 1] == pytest.approx(rad * math.sin(2 * math.pi * u2),
                                                              rel=1e-14, abs=1e-15)


def test_reaction_reset_maps_five_blocks_and_caches_the_noisy_energy():
    """x[4 sub + i] = -3 + 6 u(w_i) from RESET sub-blocks 0..4; entry 20 is
    E(x) + 0.05 z with z the cos normal of the ENV_NOISE block (t, row)."""
    from paper_2408_00930_amd import inputs
    p = inputs.reaction_params(2).astype(np.float64)
    s = O.reset_row(_env(O.REACTION, ROW + 1, params=p), SEED, EPOCH, T, ROW)
    for sub in range(5):
        w = O.draw(SEED, T, ROW, O.RESET, sub, EPOCH)
        for i in range(4):
            assert s[4 * sub + i] == -3.0 + 6.0 * _u(w[i])
    wn = O.draw(SEED, T, ROW, O.ENV_NOISE, 0, EPOCH)
    z = math.sqrt(-2.0 * math.log(_u(wn[0]))) * math.cos(2 * math.pi * _u(wn[1]))
    assert s[20] == pytest.approx(O.reaction_energy(p, s[:20]) + 0.05 * z, rel=1e-13, abs=1e-13)


# --------------------------------------------------------------- market ----

def test_market_three_agents_by_hand():
    """Actions 13, 27, 40 decode to (labour, trade) = (1/3, -1/2), (7/9, 0),
    (0, 1). Demand D = 1, supply S = 1/3 + 1/2 + 7/9 = 1.6111111111111112,
    price p = 1.001 / 1.6121111111111112 = 0.6209249431387415. Consumption:
    max(0, 1/3 - 1/2) = 0, 7/9, 1/p = 1.6105006105006106."""
    rng = np.random.default_rng(31)
    s = rng.normal(size=(3, 32))
    nxt, rew, price = O.market_step(s, [13, 27, 40])
    assert price == pytest.approx(0.6209249431387415, rel=1e-15)
    cons = [0.0, 0.7777777777777778, 1.6105006105006106]
    lab = [1 / 3, 7 / 9, 0.0]
    trade = [-0.5, 0.0, 1.0]
    for i in range(3):
        assert nxt[i, 0] == pytest.approx(0.9 * s[i, 0] + 0.1 * (cons[i] - 0.5), rel=1e-15)
        assert nxt[i, 1] == pytest.approx(-0.4765450688642452, rel=1e-14)    # log p
        assert nxt[i, 2] == pytest.approx(lab[i], rel=1e-15)
        assert nxt[i, 3] == trade[i]
        assert nxt[i, 4] == pytest.approx(cons[i], rel=1e-15)
    # log(1 + c) - 0.1 labour^2
    assert rew == pytest.approx([-0.01111111111111111, 0.514870317743068, 0.9595420077319211],
                                rel=1e-14)


# ---------------------------------------------------------- observations ----

def test_observation_encodings_at_special_angles():
    assert np.array_equal(O.observe(O.CARTPOLE, [0.1, -0.2, 0.3, -0.4]), [0.1, -0.2, 0.3, -0.4])
    # Pendulum (cos theta, sin theta, rate) at theta = pi / 3
    o = O.observe(O.PENDULUM, [math.pi / 3, -1.25])
    assert o == pytest.approx([0.5, math.sqrt(3) / 2, -1.25], abs=1e-15)
    # Acrobot (cos t1, sin t1, cos t2, sin t2, w1, w2) at t1 = pi / 2, t2 = -pi / 6
    o = O.observe(O.ACROBOT, [math.pi / 2, -math.pi / 6, 2.5, -7.0])
    assert o == pytest.approx([0.0, 1.0, math.sqrt(3) / 2, -0.5, 2.5, -7.0], abs=1e-15)
    x = np.arange(32) * 0.25 - 3.0
    assert np.array_equal(O.observe(O.MARKET, x), x)
    assert np.array_equal(O.observe(O.REACTION, np.append(x[:20], 99.0)), x[:20])


# ------------------------------------------- rounding points of the backward ----

def _bf16(t):
    import torch
    return t.to(torch.bfloat16).to(torch.float64)


@pytest.mark.parametrize("n_act", [0, 3])
def test_bf16_backward_rounds_head_grad_dz2_and_dz1(n_act):
    """One sample of a BF16 policy. Autograd in FP64 (torch) gives the loss's
    gradient with respect to the head; the oracle must round it to BF16 before
    it meets h2 (dW3 = bf16(dh) h2^T) but not in the bias gradient; dz2 is
    W3^T bf16(dh) times tanh'(z2), rounded before W2 and h1; dz1 likewise."""
    import torch
    rng = np.random.default_rng(40 + n_act)
    d_in, h, n_head = 3, 16, (n_act if n_act else 1) + 1
    w = [O.round_bf16(rng.normal(0, s, shape)) for s, shape in
         ((0.6, (h, d_in)), (0.1, h), (0.3, (h, h)), (0.1, h), (0.4, (n_head, h)),
          (0.1, n_head))]
    hold = O._MlpHold("bf16", *w)
    obs = rng.normal(0, 1, (1, d_in))
    act = np.array([1.0 if n_act else 0.37])
    adv, ret = np.array([0.9]), np.array([-0.4])
    cv, ce, log_std = 0.5, 0.02, -0.3
    g = O.ac_grad(hold, n_act, obs, act, adv, ret, cv, ce, quant_backward=True,
                  log_std=np.array([log_std]))

    W1, b1, W2, b2, W3, b3 = [torch.tensor(a, dtype=torch.float64) for a in w]
    x0 = _bf16(torch.tensor(obs[0]))
    t1 = torch.tanh(W1 @ x0 + b1)
    x1 = _bf16(t1)
    t2 = torch.tanh(W2 @ x1 + b2)
    x2 = _bf16(t2)
    head = (W3 @ x2 + b3).requires_grad_(True)
    v = head[-1]
    if n_act:
        lg = head[:n_act]
        logp = torch.log_softmax(lg, 0)[int(act[0])]
        p = torch.softmax(lg, 0)
        ent = -(p * torch.log(p)).sum()
    else:
        sigma = math.exp(log_std)
        logp = -0.5 * ((act[0] - head[0]) / sigma) ** 2 - log_std - 0.5 * math.log(2 * math.pi)
        ent = torch.tensor(0.0, dtype=torch.float64)
    loss = -adv[0] * logp + 0.5 * cv * (v - ret[0]) ** 2 - ce * ent
    (dh,) = torch.autograd.grad(loss, head)
    dh = dh.detach()

    assert np.allclose(g["b3"], dh.numpy(), rtol=1e-12, atol=1e-15)      # unrounded
    dhq = _bf16(dh)
    assert not torch.equal(dhq, dh)                                     # rounding matters here
    assert np.array_equal(g["w3"], torch.outer(dhq, x2).numpy())
    dz2 = (W3.T @ dhq) * (1 - t2 * t2)
    assert np.allclose(g["b2"], dz2.numpy(), rtol=1e-12, atol=1e-16)
    assert np.array_equal(g["w2"], torch.outer(_bf16(dz2), x1).numpy())
    dz1 = (W2.T @ _bf16(dz2)) * (1 - t1 * t1)
    assert np.allclose(g["b1"], dz1.numpy(), rtol=1e-12, atol=1e-16)
    assert np.array_equal(g["w1"], torch.outer(_bf16(dz1), x0).numpy())

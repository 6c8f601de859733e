"""Pins of the oracle's environment dynamics.

Classic control: the accelerations are checked against Euler-Lagrange
equations generated numerically from kinetic and potential energies of the
rigid bodies (tests/lagrangian.py), plus equilibria, symmetries, thresholds
and energy conservation. Market and reaction: special cases with closed
forms, permutation equivariance and an accounting identity.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle as O
from lagrangian import Body
from paper_2408_00930_amd import inputs

# constants of the project's environment specification
CP = dict(g=9.8, M=1.0, m=0.1, l=0.5, F=10.0, dt=0.02, x_lim=2.4, th_lim=12 * 2 * np.pi / 360)
PD = dict(g=10.0, m=1.0, l=1.0, dt=0.05, max_speed=8.0, max_torque=2.0)
AC = dict(l1=1.0, lc1=0.5, lc2=0.5, m1=1.0, m2=1.0, I1=1.0, I2=1.0, g=9.8, dt=0.2)


def _env(kind, n=1, offsets=None, params=None):
    return O.env_hold(kind, n, offsets, params)


# ------------------------------------------------------------- CartPole ----

def cartpole_body():
    # q = (x, theta): cart at (x, 0); uniform pole of length 2l centred at
    # (x + l sin th, l cos th), rotating with angle th; gravity along -y.
    l = CP["l"]
    return Body(
        masses=[(CP["M"], lambda q: np.array([q[0], 0 * q[0]])),
                (CP["m"], lambda q: np.array([q[0] + l * np.sin(q[1]), l * np.cos(q[1])]))],
        inertias=[(CP["m"] * (2 * l) ** 2 / 12.0, lambda q: q[1])],
        g_vec=[0.0, -CP["g"]])


def test_cartpole_accel_matches_lagrangian():
    body = cartpole_body()
    rng = np.random.default_rng(0)
    for _ in range(40):
        s = np.array([rng.uniform(-2, 2), rng.normal(), rng.uniform(-1.5, 1.5), rng.normal(0, 2)])
        for force in (CP["F"], -CP["F"]):
            want = body.accel(s[[0, 2]], s[[1, 3]], [force, 0.0])
            xdd, thdd = O.cartpole_accel(s, force)
            assert np.allclose([xdd, thdd], want, rtol=1e-7, atol=1e-8)


def test_cartpole_step_is_explicit_euler():
    env = _env(O.CARTPOLE)
    s = np.array([0.1, -0.3, 0.05, 0.4])
    for a, force in ((1, CP["F"]), (0, -CP["F"])):
        nxt, r, done, _ = O.env_step_row(env, s, a)
        xdd, thdd = O.cartpole_accel(s, force)
        assert np.allclose(nxt, s + CP["dt"] * np.array([s[1], xdd, s[3], thdd]), rtol=0,
                           atol=1e-15)
        assert r == 1.0 and not done


def test_cartpole_push_direction():
    """From rest upright, pushing right accelerates the cart right and tips
    the pole left (theta decreases)."""
    xdd, thdd = O.cartpole_accel(np.zeros(4), CP["F"])
    assert xdd > 0 and thdd < 0


def test_cartpole_mirror_symmetry():
    env = _env(O.CARTPOLE)
    rng = np.random.default_rng(1)
    for _ in range(20):
        s = rng.normal(0, 0.1, 4)
        n1, *_ = O.env_step_row(env, s, 1)
        n0, *_ = O.env_step_row(env, -s, 0)
        assert np.allclose(n1, -n0, atol=1e-15)


@pytest.mark.parametrize("which", ["x", "theta"])
@pytest.mark.parametrize("side", [1.0, -1.0])
def test_cartpole_thresholds(which, side):
    env = _env(O.CARTPOLE)
    eps = 1e-9
    for delta, want in ((-eps, False), (eps, True)):
        s = np.zeros(4)
        if which == "x":
            target = side * (CP["x_lim"] + delta)
            s[1] = target / CP["dt"]          # x' = x + dt * xdot = target
        else:
            target = side * (CP["th_lim"] + delta)
            s[3] = target / CP["dt"]
        nxt, r, done, margin = O.env_step_row(env, s, 1)
        assert done == want
        assert margin == pytest.approx(eps, abs=1e-12)
        assert r == 1.0                       # a terminal step still pays


# ------------------------------------------------------------- Pendulum ----

def pendulum_body():
    # rod of length l pivoted at the origin, theta from upright
    l = PD["l"]
    return Body(
        masses=[(PD["m"], lambda q: np.array([0.5 * l * np.sin(q[0]), 0.5 * l * np.cos(q[0])]))],
        inertias=[(PD["m"] * l**2 / 12.0, lambda q: q[0])],
        g_vec=[0.0, -PD["g"]])


def test_pendulum_accel_matches_lagrangian():
    body = pendulum_body()
    rng = np.random.default_rng(2)
    for _ in range(40):
        th, thd, u = rng.uniform(-4, 4), rng.normal(), rng.uniform(-2, 2)
        want = body.accel([th], [thd], [u])[0]
        assert O.pendulum_accel(th, u) == pytest.approx(want, rel=1e-7, abs=1e-8)


def test_pendulum_equilibria_and_reward():
    assert O.pendulum_accel(0.0, 0.0) == 0.0
    assert abs(O.pendulum_accel(np.pi, 0.0)) < 1e-14
    env = _env(O.PENDULUM)
    nxt, r, done, _ = O.env_step_row(env, [0.0, 0.0], 0.0)
    assert r == 0.0 and not done and np.array_equal(nxt, [0.0, 0.0])


def test_pendulum_semi_implicit_euler_and_clipping():
    env = _env(O.PENDULUM)
    s = np.array([0.4, 1.5])
    nxt, r, _, _ = O.env_step_row(env, s, 5.0)         # torque clipped to 2
    nxt2, r2, _, _ = O.env_step_row(env, s, 2.0)
    assert np.array_equal(nxt, nxt2) and r == r2
    w = s[1] + PD["dt"] * O.pendulum_accel(s[0], 2.0)
    assert nxt[1] == pytest.approx(w, abs=1e-15)
    assert nxt[0] == pytest.approx(s[0] + PD["dt"] * w, abs=1e-15)  # uses the new rate
    fast, *_ = O.env_step_row(env, [0.1, 7.99], 2.0)
    assert fast[1] == PD["max_speed"]


def test_wrap_angle():
    rng = np.random.default_rng(3)
    for th in rng.uniform(-50, 50, 200):
        w = O.wrap_angle(th)
        assert -np.pi <= w < np.pi
        assert np.cos(w) == pytest.approx(np.cos(th), abs=1e-12)
        assert np.sin(w) == pytest.approx(np.sin(th), abs=1e-12)


# -------------------------------------------------------------- Acrobot ----

def acrobot_body():
    # theta1 from hanging down, theta2 relative to link 1
    c = AC

    def p1(q):
        return np.array([c["lc1"] * np.sin(q[0]), -c["lc1"] * np.cos(q[0])])

    def p2(q):
        return np.array([c["l1"] * np.sin(q[0]) + c["lc2"] * np.sin(q[0] + q[1]),
                         -c["l1"] * np.cos(q[0]) - c["lc2"] * np.cos(q[0] + q[1])])
    return Body(masses=[(c["m1"], p1), (c["m2"], p2)],
                inertias=[(c["I1"], lambda q: q[0]), (c["I2"], lambda q: q[0] + q[1])],
                g_vec=[0.0, -c["g"]])


def test_acrobot_deriv_matches_lagrangian():
    body = acrobot_body()
    rng = np.random.default_rng(4)
    for _ in range(40):
        s = np.array([rng.uniform(-np.pi, np.pi), rng.uniform(-np.pi, np.pi),
                      rng.normal(0, 3), rng.normal(0, 5)])
        tau = rng.uniform(-1, 1)
        want = body.accel(s[:2], s[2:], [0.0, tau])
        got = O.acrobot_deriv(s, tau)
        assert np.allclose(got[:2], s[2:], rtol=0, atol=0)
        assert np.allclose(got[2:], want, rtol=1e-7, atol=1e-7)


def test_acrobot_step_matches_ode_solution():
    """One step integrates the Lagrangian dynamics over dt = 0.2 with a
    fourth-order error (checked against a tight adaptive solver)."""
    body = acrobot_body()
    env = _env(O.ACROBOT)
    rng = np.random.default_rng(5)
    for _ in range(8):
        s = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5),
                      rng.normal(0, 0.5), rng.normal(0, 0.5)])
        tau = rng.uniform(-1, 1)
        sol = solve_ivp(lambda t, y: np.concatenate([y[2:], body.accel(y[:2], y[2:], [0, tau])]),
                        (0, AC["dt"]), s, rtol=1e-11, atol=1e-12)
        want = sol.y[:, -1]
        nxt, r, done, _ = O.env_step_row(env, s, tau)
        err = np.abs(nxt - want).max()
        k1 = O.acrobot_deriv(s, tau)
        midpoint = s + AC["dt"] * O.acrobot_deriv(s + 0.5 * AC["dt"] * k1, tau)
        err2 = np.abs(midpoint - want).max()      # a second-order method's error
        assert err < 1e-3 and err < 0.1 * err2


def test_acrobot_energy_conserved_without_torque():
    body = acrobot_body()
    env = _env(O.ACROBOT)
    s = np.array([0.8, -0.4, 0.3, -0.2])
    e0 = body.energy(s[:2], s[2:])
    for _ in range(5):
        s, *_ = O.env_step_row(env, s, 0.0)
    assert body.energy(s[:2], s[2:]) == pytest.approx(e0, abs=5e-3)


def test_acrobot_rest_states_and_termination():
    env = _env(O.ACROBOT)
    nxt, r, done, _ = O.env_step_row(env, [0.0, 0.0, 0.0, 0.0], 0.0)   # hanging at rest
    assert np.array_equal(nxt, np.zeros(4)) and r == -1.0 and not done
    up = [np.pi - 1e-12, 0.0, 0.0, 0.0]                                 # balanced upright
    nxt, r, done, margin = O.env_step_row(env, up, 0.0)
    assert done and r == 0.0 and margin == pytest.approx(1.0, abs=1e-6)


def test_acrobot_torque_clipped():
    env = _env(O.ACROBOT)
    s = [0.1, 0.2, 0.3, 0.4]
    assert np.array_equal(O.env_step_row(env, s, 3.0)[0], O.env_step_row(env, s, 1.0)[0])


# --------------------------------------------------------------- Market ----

def test_market_decode_covers_grid():
    pairs = {O.market_decode(a) for a in range(50)}
    want = {(i / 9.0, t) for i in range(10) for t in (-1.0, -0.5, 0.0, 0.5, 1.0)}
    assert len(pairs) == 50
    assert all(any(abs(p[0] - w[0]) < 1e-15 and p[1] == w[1] for w in want) for p in pairs)


def test_market_autarky():
    """With no trade, each agent consumes its own labour."""
    rng = np.random.default_rng(6)
    s = rng.normal(size=(7, 32))
    acts = [20 + i for i in range(7)]           # trade index 2 -> tau = 0
    nxt, rew, price = O.market_step(s, acts)
    for i, a in enumerate(acts):
        l = (a % 10) / 9.0
        assert rew[i] == pytest.approx(np.log1p(l) - 0.1 * l * l, abs=1e-15)
        assert nxt[i, 4] == pytest.approx(l, abs=1e-15)


def test_market_permutation_equivariance():
    rng = np.random.default_rng(7)
    s = rng.normal(size=(23, 32))
    acts = rng.integers(0, 50, 23)
    nxt, rew, price = O.market_step(s, acts)
    perm = rng.permutation(23)
    nxt_p, rew_p, price_p = O.market_step(s[perm], acts[perm])
    assert price_p == pytest.approx(price, rel=1e-14)
    assert np.allclose(nxt_p, nxt[perm], atol=1e-14) and np.allclose(rew_p, rew[perm], atol=1e-14)


def test_market_clearing_identity():
    """Goods bought at price p = (D+eps)/(S+eps) add up to
    S + eps (D - S)/(D + eps): trade clears up to the eps guard."""
    rng = np.random.default_rng(8)
    eps = 1e-3
    for _ in range(50):
        n = int(rng.integers(1, 40))
        acts = rng.integers(0, 50, n)
        lab = np.array([O.market_decode(a)[0] for a in acts])
        tr = np.array([O.market_decode(a)[1] for a in acts])
        D, S = np.maximum(tr, 0).sum(), (lab + np.maximum(-tr, 0)).sum()
        _, _, price = O.market_step(np.zeros((n, 32)), acts)
        bought = (np.maximum(tr, 0) / price).sum()
        assert bought == pytest.approx(S + eps * (D - S) / (D + eps), rel=1e-12, abs=1e-12)


def test_market_state_decay():
    rng = np.random.default_rng(9)
    s = rng.normal(size=(5, 32))
    acts = rng.integers(0, 50, 5)
    cur = s
    for _ in range(10):
        cur, _, _ = O.market_step(cur, acts)
    assert np.allclose(cur[:, 5:], s[:, 5:] * 0.99**10, rtol=1e-13)


# ------------------------------------------------------------- Reaction ----

def _params(A=None, centres=None, widths=None, amps=None):
    d, g = inputs.RX_DIM, inputs.RX_NG
    A = np.zeros((d, d)) if A is None else A
    centres = np.zeros((g, d)) if centres is None else centres
    widths = np.ones(g) if widths is None else widths
    amps = np.zeros(g) if amps is None else amps
    return np.concatenate([A.ravel(), centres.ravel(), widths, amps])


def test_reaction_quadratic_via_eigendecomposition():
    p = inputs.reaction_params(0).astype(np.float64)
    A = p[:400].reshape(20, 20)
    lam, Q = np.linalg.eigh(A)
    assert lam.min() >= 0.1 - 1e-6 and lam.max() <= 2.0 + 1e-6
    quad_only = _params(A=A)
    rng = np.random.default_rng(10)
    for _ in range(20):
        x = rng.uniform(-3, 3, 20)
        assert O.reaction_energy(quad_only, x) == pytest.approx(0.5 * np.sum(lam * (Q.T @ x) ** 2),
                                                                rel=1e-12)


def test_reaction_gaussian_bumps():
    rng = np.random.default_rng(11)
    centres = rng.uniform(-3, 3, (64, 20))
    amps = np.zeros(64)
    amps[17] = 1.7
    widths = np.full(64, 0.6)
    p = _params(centres=centres, widths=widths, amps=amps)
    assert O.reaction_energy(p, centres[17]) == pytest.approx(1.7, rel=1e-14)
    x = centres[17].copy()
    x[3] += 0.6                                  # one width away: e^{-1/2}
    assert O.reaction_energy(p, x) == pytest.approx(1.7 * np.exp(-0.5), rel=1e-14)


def test_reaction_step_moves_one_coordinate_and_pays_energy_drop():
    p = inputs.reaction_params(0).astype(np.float64)
    env = _env(O.REACTION, 1, params=p)
    s0 = O.reset_row(env, seed=5, epoch=0, t=0, row=3)
    for a in (0, 1, 7, 38, 39):
        nxt, r, done, _ = O.env_step_row(env, s0, a, seed=5, epoch=0, t=0, row=3)
        dx = nxt[:20] - s0[:20]
        assert np.count_nonzero(dx) == 1 and np.argmax(np.abs(dx)) == a // 2
        assert dx[a // 2] == pytest.approx(0.05 if a % 2 == 0 else -0.05, abs=1e-15)
        assert r == pytest.approx(-(nxt[20] - s0[20]), abs=1e-15) and not done


def test_reaction_noise_only_potential():
    """With a flat potential the cached energy is pure noise 0.05 * xi."""
    env = _env(O.REACTION, 1, params=_params())
    s = O.reset_row(env, seed=9, epoch=2, t=4, row=1)
    w = O.draw(9, 4, 1, O.ENV_NOISE, 0, 2)
    z, _ = O.box_muller(O.u01(w[0]), O.u01(w[1]))
    assert s[20] == pytest.approx(0.05 * z, abs=1e-15)
    assert np.all((s[:20] > -3) & (s[:20] < 3))

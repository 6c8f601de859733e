"""User environment kinds compiled at run time (wsx_user_kind_register).

Copies of the built-in Pendulum (BF16 policy, Gaussian head) and CartPole
(FP32 policy, categorical head) registered as user code must roll out
exactly as the built-in kinds do on the kernel of the same shape (the same
templates, the same arithmetic); a new environment (a point mass) is checked
step by step against a numpy re-implementation of its source."""
import numpy as np
import pytest

import user_envs
from gpu_cases import say
from paper_2408_00930_amd import inputs

pytestmark = pytest.mark.gpu


def _wsx():
    from paper_2408_00930_amd import wsx
    return wsx


_KINDS = {}


def _kind(name):
    wsx = _wsx()
    if name not in _KINDS:
        say("register user kind", name)
        if name == "pendulum":
            _KINDS[name] = wsx.user_kind_register(user_envs.PENDULUM, 2, 3, 0, "bf16", 256)
        elif name == "cartpole":
            _KINDS[name] = wsx.user_kind_register(user_envs.CARTPOLE, 4, 4, 2, "f32", 64)
        elif name == "group_walk":
            _KINDS[name] = wsx.user_kind_register(user_envs.GROUP_WALK, 4, 4, 0, "bf16", 256)
        else:
            _KINDS[name] = wsx.user_kind_register(user_envs.POINT_MASS, 2, 2, 0, "bf16", 256)
    return _KINDS[name]


def _roll(kind, n, T, pol_kind, dtype, hidden, mode=0, chunk=None, **shape):
    wsx = _wsx()
    env = wsx.Env(kind, n, seed=5, **shape)
    dp = wsx.DevicePolicy(inputs.policy_for(pol_kind, dtype, hidden, seed=1))
    tr = wsx.Trajectory(kind, T, env.rows)
    if chunk is not None:
        env.set_chunk(chunk)
    wsx.env_reset(env, 2)
    wsx.rollout(env, dp, T, tr, mode)
    out = tr.host()
    out["state"] = env.state.cpu().numpy().copy()
    return out


@pytest.mark.parametrize("name,builtin,dtype,hidden,shape",
                         [("pendulum", 2, "bf16", 256, dict(tile_rows=80, waves=8, occupancy=2)),
                          ("cartpole", 1, "f32", 64, dict(tile_rows=16, waves=4, occupancy=1))])
def test_user_copy_of_a_builtin_kind_is_bitwise_equal(name, builtin, dtype, hidden, shape):
    wsx = _wsx()
    k = _kind(name)
    assert k >= 100
    T = 37
    say("user kind vs builtin", name)
    ref = _roll(builtin, 333, T, builtin, dtype, hidden, **shape)
    got = _roll(k, 333, T, builtin, dtype, hidden)
    for f in ref:
        assert np.array_equal(got[f], ref[f]), f
    # the chunked graph mode runs the loaded kernel inside a captured graph
    g = _roll(k, 333, T, builtin, dtype, hidden, mode=wsx.MODE_FUSED_GRAPH, chunk=10)
    for f in ref:
        assert np.array_equal(g[f], ref[f]), f


def test_user_kind_rejects_the_plain_modes():
    wsx = _wsx()
    k = _kind("pendulum")
    env = wsx.Env(k, 20, seed=0)
    dp = wsx.DevicePolicy(inputs.policy_for(2, "bf16", 256, seed=0))
    tr = wsx.Trajectory(k, 3, env.rows)
    wsx.env_reset(env, 0)
    with pytest.raises(wsx.WsxError, match="fused modes only"):
        wsx.rollout(env, dp, 3, tr, wsx.MODE_PLAIN)


def test_new_user_environment_runs_as_written():
    """Point mass: every recorded transition equals the numpy step of the
    source's dynamics from the recorded observation and action."""
    wsx = _wsx()
    k = _kind("point_mass")
    say("point mass")
    T, n = 25, 300
    env = wsx.Env(k, n, seed=3)
    pol = inputs.make_policy(2, 256, 256, 1, "bf16", seed=4)
    dp = wsx.DevicePolicy(pol)
    tr = wsx.Trajectory(k, T, env.rows)
    wsx.env_reset(env, 1)
    wsx.rollout(env, dp, T, tr)
    g = tr.host()
    obs, act = g["obs"].astype(np.float32), g["action"].astype(np.float32)
    assert np.isfinite(obs).all() and np.isfinite(g["value"]).all()
    assert (np.abs(obs[0]) <= 1.0).all()                     # reset range
    # the device contracts a * b + c into one FMA where numpy rounds twice:
    # within one FP32 rounding of the values involved
    def close(a, b):
        return np.abs(a - b) <= 2e-7 + 2e-6 * np.abs(b)
    for t in range(T - 1):
        x2, v2, r, d = user_envs.point_mass_step(obs[t, :, 0], obs[t, :, 1], act[t])
        sure = np.abs(np.abs(x2) - 2.0) > 1e-5                 # not at the threshold
        assert np.array_equal(g["done"][t].astype(bool)[sure], d[sure]), t
        assert close(g["reward"][t], r).all(), t
        live = ~g["done"][t].astype(bool)                      # terminated rows restart
        assert close(obs[t + 1, live, 0], x2[live]).all(), t
        assert close(obs[t + 1, live, 1], v2[live]).all(), t


def test_user_kind_sets_batch_in_one_launch():
    """Two sets of the user Pendulum with their own policies in one
    wsx_rollout_batch launch equal the built-in Pendulum rolled out alone."""
    wsx = _wsx()
    k = _kind("pendulum")
    say("user kind batch")
    T = 19
    ref, sets = [], []
    for n, seed, pseed in ((357, 11, 1), (64, 13, 3)):
        env = wsx.Env(2, n, seed=seed, tile_rows=80, waves=8, occupancy=2)
        dp = wsx.DevicePolicy(inputs.policy_for(2, "bf16", 256, seed=pseed))
        tr = wsx.Trajectory(2, T, env.rows)
        wsx.env_reset(env, 4)
        wsx.rollout(env, dp, T, tr)
        ref.append(tr.host())
        sets.append((wsx.Env(k, n, seed=seed), dp))
    trs = [wsx.Trajectory(k, T, env.rows) for env, _ in sets]
    for env, _ in sets:
        wsx.env_reset(env, 4)
    wsx.rollout_batch([e for e, _ in sets], [p for _, p in sets], T, trs)
    for i, tr in enumerate(trs):
        got = tr.host()
        for f in got:
            assert np.array_equal(got[f], ref[i][f]), (i, f)


def test_user_kind_served_with_builtin_requests():
    """A request of the user Pendulum served in a mix with built-in Pendulum
    and Acrobot requests returns the built-in Pendulum's direct results."""
    import torch
    wsx = _wsx()
    k = _kind("pendulum")
    say("user kind served")
    dp = wsx.DevicePolicy(inputs.policy_for(2, "bf16", 256, seed=7))
    acro = wsx.DevicePolicy(inputs.policy_for(3, "bf16", 256, seed=8))
    T, n = 45, 150
    env = wsx.Env(2, n, seed=5)
    tr = wsx.Trajectory(2, T, env.rows)
    wsx.env_reset(env, 2)
    wsx.rollout(env, dp, T, tr)
    ret, adv = wsx.compute_returns(tr, T, 0.99, 0.95, True, torch.float32)
    want = tr.host()
    want["returns"], want["advantages"] = ret.cpu().numpy(), adv.cpu().numpy()
    srv = wsx.Server(1 << 30, chunk_steps=16, max_batch=32)
    others = [srv.submit(kind=2, policy=dp, horizon=30, n_envs=90, seed=11),
              srv.submit(kind=3, policy=acro, horizon=60, n_envs=200, seed=12)]
    rid = srv.submit(kind=k, policy=dp, horizon=T, n_envs=n, seed=5, epoch=2)
    r = srv.wait(rid, 60000)
    got = {f: v.cpu().numpy() for f, v in srv.view(r, k).items()}
    for o in others:
        srv.wait(o, 60000)
        srv.release(o)
    srv.release(rid)
    srv.close()
    for f in ("obs", "action", "reward", "done", "value", "logp", "last_value", "returns",
              "advantages"):
        assert np.array_equal(got[f], want[f]), f


def test_user_environment_with_lane_groups():
    """Four lanes per row (LANES = 4): the reward summed over the row's lanes
    with group_sum, and the state, match numpy on every transition."""
    wsx = _wsx()
    k = _kind("group_walk")
    say("group walk")
    T, n = 20, 301
    env = wsx.Env(k, n, seed=8)
    dp = wsx.DevicePolicy(inputs.make_policy(4, 256, 256, 1, "bf16", seed=9))
    tr = wsx.Trajectory(k, T, env.rows)
    wsx.env_reset(env, 0)
    wsx.rollout(env, dp, T, tr)
    g = tr.host()
    obs, act = g["obs"].astype(np.float32), g["action"].astype(np.float32)
    assert (np.abs(obs[0]) <= 1.0).all() and not g["done"].any()

    def close(a, b):
        return np.abs(a - b) <= 1e-6 + 4e-6 * np.abs(b)
    for t in range(T - 1):
        s2, r = user_envs.group_walk_step(obs[t], act[t])
        assert close(g["reward"][t], r).all(), t
        assert close(obs[t + 1], s2).all(), t

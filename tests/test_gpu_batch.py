"""Several environment sets in one fused launch (wsx_rollout_batch): each set
gets exactly what wsx_rollout gives it alone on a kernel with the same waves."""
import numpy as np
import pytest

from gpu_cases import DTYPE, HIDDEN, say
from paper_2408_00930_amd import inputs

pytestmark = pytest.mark.gpu


def _wsx():
    from paper_2408_00930_amd import wsx
    return wsx


def _set(wsx, kind, n, seed, pol_seed, **shape):
    env = wsx.Env(kind, n, seed=seed, **shape)
    dp = wsx.DevicePolicy(inputs.policy_for(kind, DTYPE[kind], HIDDEN[kind], seed=pol_seed))
    return env, dp


@pytest.mark.parametrize("shape", [dict(tile_rows=80, waves=8), dict(tile_rows=40, waves=4),
                                   dict(tile_rows=48, waves=4, occupancy=2)])
def test_pendulum_and_acrobot_in_one_launch_equal_separate(shape):
    wsx = _wsx()
    say("batch pendulum+acrobot", shape)
    T = 23
    sets = [_set(wsx, 2, 357, 11, 1, **shape), _set(wsx, 3, 1001, 12, 2, **shape),
            _set(wsx, 2, 64, 13, 3, **shape)]          # a second pendulum set, own policy
    alone = []
    for env, dp in sets:
        tr = wsx.Trajectory(env.kind, T, env.rows)
        wsx.env_reset(env, 4)
        wsx.rollout(env, dp, T, tr)
        alone.append(tr.host())
    trs = [wsx.Trajectory(env.kind, T, env.rows) for env, _ in sets]
    for env, _ in sets:
        wsx.env_reset(env, 4)
    wsx.rollout_batch([e for e, _ in sets], [p for _, p in sets], T, trs)
    for i, tr in enumerate(trs):
        got = tr.host()
        for k in got:
            assert np.array_equal(got[k], alone[i][k]), (i, k)
        assert sets[i][0].info()[1] == T


def test_batch_of_one_kind_different_policies_and_horizon_zero():
    wsx = _wsx()
    say("batch same kind")
    a = _set(wsx, 1, 100, 1, 1)
    b = _set(wsx, 1, 33, 2, 2)
    for T in (0, 9):
        ref = []
        for env, dp in (a, b):
            tr = wsx.Trajectory(1, T, env.rows)
            wsx.env_reset(env, 0)
            wsx.rollout(env, dp, T, tr)
            ref.append(tr.host())
        trs = [wsx.Trajectory(1, T, env.rows) for env, _ in (a, b)]
        for env, _ in (a, b):
            wsx.env_reset(env, 0)
        wsx.rollout_batch([a[0], b[0]], [a[1], b[1]], T, trs)
        for i in range(2):
            got = trs[i].host()
            for k in got:
                assert np.array_equal(got[k], ref[i][k]), (T, i, k)


def test_batch_rejects_bad_mixes():
    wsx = _wsx()
    say("batch errors")
    p = _set(wsx, 2, 50, 1, 1)
    c = _set(wsx, 1, 50, 1, 1)
    tr = lambda e: wsx.Trajectory(e.kind, 4, e.rows)
    with pytest.raises(wsx.WsxError):        # cart-pole and pendulum: no such kernel
        wsx.rollout_batch([p[0], c[0]], [p[1], c[1]], 4, [tr(p[0]), tr(c[0])])
    with pytest.raises(wsx.WsxError):        # the same set twice
        wsx.rollout_batch([p[0], p[0]], [p[1], p[1]], 4, [tr(p[0]), tr(p[0])])
    five = [_set(wsx, 2, 20, s, 1) for s in range(5)]
    with pytest.raises(wsx.WsxError):        # more than four sets
        wsx.rollout_batch([e for e, _ in five], [d for _, d in five], 4, [tr(e) for e, _ in five])
    small = wsx.Trajectory(2, 2, 50)
    with pytest.raises(wsx.WsxError):        # trajectory shorter than the horizon
        wsx.rollout_batch([p[0]], [p[1]], 4, [small])

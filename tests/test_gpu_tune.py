"""The autotuner: it times real candidates, records the winner, and an
environment set created with the default shape afterwards runs on it with the
same results as one given that shape explicitly."""
import numpy as np
import pytest

from gpu_cases import DTYPE, HIDDEN, say
from paper_2408_00930_amd import inputs

pytestmark = pytest.mark.gpu


def _wsx():
    from paper_2408_00930_amd import wsx
    return wsx


def _roll(wsx, env, dp, kind, T, mode=None):
    traj = wsx.Trajectory(kind, T, env.rows)
    wsx.env_reset(env, 1)
    wsx.rollout(env, dp, T, traj, wsx.MODE_FUSED if mode is None else mode)
    return traj.host()


@pytest.mark.parametrize("kind,n", [(2, 3001), (4, 301)])
def test_autotune_records_a_shape_that_env_create_uses(kind, n):
    import torch
    wsx = _wsx()
    say("autotune", kind, n)
    dp = wsx.DevicePolicy(inputs.policy_for(kind, DTYPE[kind], HIDDEN[kind], seed=kind))
    offs = inputs.agent_offsets(n, seed=3) if kind == wsx.MARKET else None
    best = wsx.autotune(kind, n, dp, horizon=12, reps=1, seed=5, agent_offsets=offs)
    print(best, flush=True)
    assert best["tile_rows"] >= 1 and best["waves"] in (4, 8) and best["us_per_step"] > 0
    assert best["chunk_steps"] in (0, 6, 3, 2)
    rows = int(offs[-1]) if offs is not None else n
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert wsx.tune_lookup(kind, n, rows, cus) == best
    tuned = wsx.Env(kind, n, seed=5, agent_offsets=offs)
    assert wsx.env_shape(tuned) == (best["tile_rows"], best["waves"], best["occupancy"],
                                    best["chunk_steps"])
    explicit = wsx.Env(kind, n, seed=5, agent_offsets=offs, tile_rows=best["tile_rows"],
                       waves=best["waves"], occupancy=best["occupancy"])
    a = _roll(wsx, tuned, dp, kind, 12, wsx.MODE_FUSED_GRAPH)
    b = _roll(wsx, explicit, dp, kind, 12)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_autotune_batch_records_one_shape_for_the_mix():
    wsx = _wsx()
    say("autotune batch")
    pols = {k: wsx.DevicePolicy(inputs.policy_for(k, DTYPE[k], HIDDEN[k], seed=k)) for k in (2, 3)}
    spec = [dict(kind=2, n_envs=3001, policy=pols[2], seed=1),
            dict(kind=3, n_envs=2999, policy=pols[3], seed=2)]
    best = wsx.autotune_batch(spec, horizon=10, reps=1)
    print(best, flush=True)
    envs = [wsx.Env(d["kind"], d["n_envs"], seed=d["seed"]) for d in spec]
    for e in envs:
        assert wsx.env_shape(e)[:3] == (best["tile_rows"], best["waves"], best["occupancy"])
    T = 10
    trs = [wsx.Trajectory(e.kind, T, e.rows) for e in envs]
    for e in envs:
        wsx.env_reset(e, 1)
    wsx.rollout_batch(envs, [pols[2], pols[3]], T, trs)
    for e, tr, d in zip(envs, trs, spec):
        # the batched launch equals each set's own launch on the same shape
        ref = _roll(wsx, wsx.Env(d["kind"], d["n_envs"], seed=d["seed"]), pols[d["kind"]],
                    d["kind"], T)
        got = tr.host()
        for k in got:
            assert np.array_equal(got[k], ref[k]), k

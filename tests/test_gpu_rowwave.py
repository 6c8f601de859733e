"""The row-per-wave form of the FP32 64-wide policy (CartPole): one wave per
replica, lane j owning hidden feature j, FP32 FMAs, no workgroup barrier in
a step. Checked like the MFMA form: lock-step against the oracle with the
kernel's own FP32 hidden activations adopted (the head within its FP32
accumulation bound, draws excused only next to a CDF boundary and counted),
free-running against the oracle, and every execution form bitwise equal to
the fused one."""
import json

import numpy as np
import pytest

import oracle as O
from gpu_cases import Case, say
from test_gpu_parity import lockstep

pytestmark = pytest.mark.gpu

RW = dict(tile_rows=1, waves=1)


def _wsx():
    from paper_2408_00930_amd import wsx
    return wsx


def test_shape_is_the_row_per_wave_kernel():
    wsx = _wsx()
    c = Case(O.CARTPOLE, 50, seed=1, **RW)
    assert wsx.env_shape(c.env)[:2] == (1, 1)
    assert c.env.tiles() == (50, 1)


@pytest.mark.parametrize("n_envs,T", [(100, 60), (7, 30)])
def test_lockstep_matches_oracle(n_envs, T):
    c = Case(O.CARTPOLE, n_envs, seed=11, **RW)
    say("row-per-wave lock-step", n_envs, T)
    stats = {}
    n_dec, n_exc = lockstep(c, T, stats=stats)
    stats.update(kind=O.CARTPOLE, form="row per wave", rows=c.rows, steps=T, excused=n_exc,
                 decisions=n_dec)
    print("PRECISION " + json.dumps(stats), flush=True)


def test_free_running_matches_oracle():
    wsx = _wsx()
    c = Case(O.CARTPOLE, 300, seed=2, **RW)
    T = 300
    traj = wsx.Trajectory(O.CARTPOLE, T, c.rows)
    wsx.env_reset(c.env, 0)
    say("row-per-wave free-running", T)
    wsx.rollout(c.env, c.dpol, T, traj)
    g = traj.host()
    ref = O.rollout(c.ohold, c.mlp, c.seed, 0, 0, T, O.env_reset(c.ohold, c.seed, 0), c.log_std)
    diverged = 0
    for r in range(c.rows):
        bad = np.nonzero((g["action"][:, r] != ref["action"][:, r]) |
                         (g["done"][:, r] != ref["done"][:, r]))[0]
        stop = bad[0] if len(bad) else T
        if len(bad):
            t = bad[0]
            assert (ref["margin_action"][t, r] < 1e-6 or ref["margin_done"][t, r] < 1e-5 or
                    (t > 0 and ref["margin_done"][t - 1, r] < 1e-5)), (r, t)
            diverged += 1
        assert np.allclose(g["obs"][:stop, r], ref["obs"][:stop, r], rtol=1e-4, atol=1e-4)
        assert np.allclose(g["value"][:stop, r], ref["value"][:stop, r], rtol=1e-4, atol=1e-4)
        assert np.array_equal(g["reward"][:stop, r], ref["reward"][:stop, r])
    print(f"row-per-wave free-running: {diverged} of {c.rows} envs hit an excused decision",
          flush=True)
    assert diverged <= c.rows // 50


def _run(c, mode, T, epoch=3):
    wsx = _wsx()
    traj = wsx.Trajectory(c.kind, T, c.rows)
    wsx.env_reset(c.env, epoch)
    wsx.rollout(c.env, c.dpol, T, traj, mode)
    out = traj.host()
    out["state"] = c.gpu_state()
    return out


@pytest.mark.parametrize("n", [1, 70, 1500])
def test_forms_equal_fused_bitwise(n):
    """Plain per-step launches, their graph, and the horizon as chunked fused
    launches in a graph all equal one fused launch; so does a roll-out
    resumed after a split."""
    wsx = _wsx()
    c = Case(O.CARTPOLE, n, seed=4, **RW)
    say("row-per-wave forms", n)
    T = 67
    f = _run(c, wsx.MODE_FUSED, T)
    for mode in (wsx.MODE_PLAIN, wsx.MODE_GRAPH, wsx.MODE_FUSED_GRAPH):
        c.env.set_chunk(16)
        g = _run(c, mode, T)
        for k in f:
            assert np.array_equal(f[k], g[k]), (mode, k)
    # resume: 30 + 37 steps into one trajectory's two halves
    traj = wsx.Trajectory(c.kind, T, c.rows)
    a, b = wsx.Trajectory(c.kind, 30, c.rows), wsx.Trajectory(c.kind, 37, c.rows)
    wsx.env_reset(c.env, 3)
    wsx.rollout(c.env, c.dpol, 30, a)
    wsx.rollout(c.env, c.dpol, 37, b)
    ha, hb = a.host(), b.host()
    for k in ("obs", "action", "reward", "done", "value", "logp"):
        assert np.array_equal(np.concatenate([ha[k], hb[k]]), f[k]), k
    assert np.array_equal(hb["last_value"], f["last_value"])


def test_one_launch_and_batch_equal_separate_calls():
    import torch
    wsx = _wsx()
    say("row-per-wave one launch")
    sets = [Case(O.CARTPOLE, 1000, seed=5, **RW), Case(O.CARTPOLE, 333, seed=6, **RW)]
    T = 50
    sep = []
    for c in sets:
        tr = wsx.Trajectory(c.kind, T, c.rows)
        wsx.env_reset(c.env, 9)
        wsx.rollout(c.env, c.dpol, T, tr)
        r, a = wsx.compute_returns(tr, T, 0.99, 0.95, True, torch.float64)
        sep.append((tr.host(), r.cpu().numpy(), a.cpu().numpy()))
    trs = [wsx.Trajectory(c.kind, T, c.rows) for c in sets]
    ret = [torch.empty((T, c.rows), dtype=torch.float64, device="cuda") for c in sets]
    adv = [torch.empty_like(x) for x in ret]
    wsx.rollout_batch_ext([c.env for c in sets], [c.dpol for c in sets], T, trs, epoch=9,
                          returns=ret, advantages=adv, gamma=0.99, lam=0.95)
    torch.cuda.synchronize()
    for i, c in enumerate(sets):
        got = trs[i].host()
        for k in got:
            assert np.array_equal(got[k], sep[i][0][k]), (i, k)
        for x, y in ((ret[i].cpu().numpy(), sep[i][1]), (adv[i].cpu().numpy(), sep[i][2])):
            assert np.max(np.abs(x - y) / np.maximum(1.0, np.abs(y))) <= 1e-12

"""wsx_ac_grad_static (no workspace argument, nothing allocated by the
library: the workspace is the library's static device array) against
wsx_ac_grad with a caller-owned workspace, through the C ABI: the gradients
are equal bit for bit (the same kernels and partial-sum layout), on two calls
in a row, the second over fewer samples; counts past the bound are
rejected."""
import numpy as np
import pytest

import oracle as O
from gpu_cases import DTYPE, HIDDEN, say
from paper_2408_00930_amd import inputs

pytestmark = pytest.mark.gpu


def _samples(kind, n_envs, T, seed):
    import torch
    from paper_2408_00930_amd import wsx
    pol = inputs.policy_for(kind, DTYPE[kind], HIDDEN[kind], seed=seed)
    offs = inputs.agent_offsets(n_envs, seed=seed) if kind == O.MARKET else None
    env = wsx.Env(kind, n_envs, seed=seed, agent_offsets=offs)
    dp = wsx.DevicePolicy(pol)
    tr = wsx.Trajectory(kind, T, env.rows)
    wsx.env_reset(env, 2)
    wsx.rollout(env, dp, T, tr)
    ret, adv = wsx.compute_returns(tr, T, inputs.GAMMA, inputs.LAMBDA, True, torch.float32)
    torch.cuda.synchronize()
    return (dp, tr.obs.reshape(-1, pol.d_in), tr.action.reshape(-1), ret.reshape(-1),
            adv.reshape(-1))


@pytest.mark.parametrize("kind,n_envs,T", [(O.PENDULUM, 1024, 2), (O.CARTPOLE, 700, 3),
                                           (O.MARKET, 45, 1)])
def test_static_gradient_equals_the_workspace_gradient(kind, n_envs, T):
    import torch
    from paper_2408_00930_amd import wsx
    dp, obs, act, ret, adv = _samples(kind, n_envs, T, seed=kind)
    n_act = wsx.N_ACTIONS[kind]
    top = min(wsx.AC_STATIC_MAX_SAMPLES, ret.numel())
    for n in (top, 333):
        say("no-alloc gradient", kind, n)
        args = (obs[:n].contiguous(), act[:n].contiguous(), ret[:n].contiguous(),
                adv[:n].contiguous())
        want = wsx.ac_grad(dp, n_act, *args, 0.5, 0.01)
        got = wsx.ac_grad_static(dp, n_act, *args, 0.5, 0.01)
        torch.cuda.synchronize()
        names = wsx.Grads.NAMES if n_act == 0 else wsx.Grads.NAMES[:-1]
        for k in names:
            assert torch.equal(got[k], want[k]), (kind, n, k)
            assert torch.isfinite(got[k]).all()


def test_static_gradient_rejects_more_samples_than_its_workspace_holds():
    import torch
    from paper_2408_00930_amd import wsx
    dp, obs, act, ret, adv = _samples(O.PENDULUM, 1100, 2, seed=1)
    n = wsx.AC_STATIC_MAX_SAMPLES + 1
    assert ret.numel() >= n
    say("no-alloc gradient past the bound")
    with pytest.raises(wsx.WsxError, match="at most"):
        wsx.ac_grad_static(dp, 0, obs[:n].contiguous(), act[:n].contiguous(),
                           ret[:n].contiguous(), adv[:n].contiguous())
    torch.cuda.synchronize()

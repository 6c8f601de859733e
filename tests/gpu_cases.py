"""Shared set-up of the GPU parity tests: seeded inputs for both sides, the
device objects, and the comparison helpers. The oracle and the HIP path
share only the inputs drawn here (paper_2408_00930_amd.inputs)."""
import sys

import numpy as np

import oracle as O
from paper_2408_00930_amd import inputs

HIDDEN = {O.CARTPOLE: 64, O.PENDULUM: 256, O.ACROBOT: 256, O.MARKET: 256, O.REACTION: 512}
DTYPE = {O.CARTPOLE: "f32", O.PENDULUM: "bf16", O.ACROBOT: "bf16", O.MARKET: "bf16",
         O.REACTION: "fp8"}


def say(*args):
    """Name the case before a GPU step (flushed, so it survives a crash)."""
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


class Case:
    def __init__(self, kind, n_envs, seed=0, tile_rows=0, offsets=None):
        from paper_2408_00930_amd import wsx
        self.kind = kind
        self.seed = seed
        self.policy = inputs.policy_for(kind, DTYPE[kind], HIDDEN[kind], seed=seed)
        if kind == O.MARKET and offsets is None:
            offsets = inputs.agent_offsets(n_envs, seed=seed)
        self.offsets = offsets
        self.params = inputs.reaction_params(seed) if kind == O.REACTION else None
        self.env = wsx.Env(kind, n_envs, seed=seed, agent_offsets=offsets, params=self.params,
                           tile_rows=tile_rows)
        self.dpol = wsx.DevicePolicy(self.policy)
        self.rows = self.env.rows
        self.ohold = O.env_hold(kind, n_envs, offsets,
                                None if self.params is None else self.params.astype(np.float64))
        self.mlp = O.mlp_hold(self.policy)
        self.log_std = self.policy.exact("log_std")

    def gpu_state(self):
        """[rows, state_dim] float64 copy of the device state."""
        return self.env.state.cpu().numpy().T.astype(np.float64).copy()

    def set_gpu_state(self, st):
        import torch
        self.env.state.copy_(torch.from_numpy(np.ascontiguousarray(st.T, np.float32)))


def env_groups(case):
    """Row ranges of the environments (one row each except the market)."""
    if case.kind == O.MARKET:
        off = case.offsets
        return [(int(off[e]), int(off[e + 1])) for e in range(len(off) - 1)]
    return [(r, r + 1) for r in range(case.rows)]

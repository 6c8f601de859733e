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
    def __init__(self, kind, n_envs, seed=0, tile_rows=0, offsets=None, waves=0):
        from paper_2408_00930_amd import wsx
        self.kind = kind
        self.seed = seed
        self.policy = inputs.policy_for(kind, DTYPE[kind], HIDDEN[kind], seed=seed)
        if kind == O.MARKET and offsets is None:
            offsets = inputs.agent_offsets(n_envs, seed=seed)
        self.offsets = offsets
        self.params = inputs.reaction_params(seed) if kind == O.REACTION else None
        self.env = wsx.Env(kind, n_envs, seed=seed, agent_offsets=offsets, params=self.params,
                           tile_rows=tile_rows, waves=waves)
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


def adopted_head(env, dpol, policy, obs):
    """Head outputs of the roll-out kernel of `env` for observations obs
    [n, d_in] (float32), checked against the oracle with the device's
    rounding decisions adopted.

    The trace kernel (the roll-out's own MLP code and shape) gives the
    quantised hidden-layer codes. A code that differs from the oracle's FP64
    rounding must lie within the FP32 error bound of the deciding midpoint (a
    counted flip); the oracle then evaluates the next layer from the device's
    code, and the head from the device's layer-2 codes in FP64, and the
    device's head must lie within the head's own accumulation bound (FP32:
    gamma_{K+16} sum|W3 h2| + u |y|; FP8 adds the matrix core's group
    truncation). Returns (device head, adoption result, bound, error)."""
    import torch
    from paper_2408_00930_amd import wsx
    obs = np.ascontiguousarray(obs, np.float32)
    head_t, h1, h2 = wsx.policy_trace(env, dpol, torch.from_numpy(obs).cuda())
    head_t = head_t.cpu().numpy().astype(np.float64)
    ad = O.mlp_adopt(policy, obs.astype(np.float64), h1, h2)
    bad = np.nonzero(ad["ratio"] > 1.0)
    assert len(bad[0]) == 0, f"codes far from any midpoint: rows {bad[0][:5]}, ratio " \
                             f"{ad['ratio'][bad][:5]}"
    bound = ad["head_bound"]
    err = np.abs(head_t - ad["head"])
    worst = np.nonzero(err > bound)
    assert len(worst[0]) == 0, f"head beyond its FP32 bound: rows {worst[0][:5]}, err " \
                               f"{err[worst][:5]}, bound {bound[worst][:5]}"
    return head_t, ad, bound, err


def flip_stats(ad, err, bound, stats):
    """Accumulate the flip counts and error figures of one adopted check."""
    cur = {"rows_checked": int(ad["flips"].shape[0]),
           "rows_with_flips": int((ad["flips"].sum(axis=1) > 0).sum()),
           "flips_h1": int(ad["flips"][:, 0].sum()), "flips_h2": int(ad["flips"][:, 1].sum())}
    for k, v in cur.items():
        stats[k] = stats.get(k, 0) + v
    for k, v in (("max_flip_ratio", ad["ratio"].max(initial=0.0)),
                 ("head_err_max", err.max(initial=0.0)),
                 ("head_err_over_bound", (err / np.maximum(bound, 1e-300)).max(initial=0.0))):
        stats[k] = max(stats.get(k, 0.0), float(v))


def check_policy_step(env, dpol, policy, kind, obs, value, action, logp, seed, epoch, t, rows,
                      log_std=None, stats=None):
    """Every row's policy results of one roll-out step against the oracle with
    the device's rounding decisions adopted (adopted_head).

    obs [n, d_in] (the recorded FP32 observations), value / action / logp [n]
    (the recorded results), rows: the rows' global indices (their Philox
    counters). The trace kernel's value must equal the recorded value bit for
    bit (it is the same code). Actions: equal, except a categorical draw
    within 2 max|logit error| + 1e-6 of a CDF boundary (the logit errors
    move the CDF by at most twice their largest; counted); log-probabilities
    within 2 max|logit error| + 2e-5; Gaussian actions within the mean's
    bound + 1e-5 and log-densities within 1e-4 (the FP32 normal draw).
    Returns the number of excused draws."""
    head_t, ad, bound, err = adopted_head(env, dpol, policy, obs)
    assert np.array_equal(head_t[:, -1], np.asarray(value, np.float64)), \
        "the trace kernel's value differs from the roll-out's"
    st = stats if stats is not None else {}
    flip_stats(ad, err, bound, st)
    n_act = O.n_actions(kind)
    a, lp, mg = O.sample_rows(ad["head"], n_act, log_std, seed, t, rows, epoch)
    action = np.asarray(action, np.float64)
    logp = np.asarray(logp, np.float64)
    if n_act:
        lb = bound[:, :n_act].max(axis=1)
        diff = a != action
        excused = int(diff.sum())
        bad = np.nonzero(diff & ~(mg < 2 * lb + 1e-6))[0]
        assert len(bad) == 0, f"rows {np.asarray(rows)[bad][:5]}: actions {action[bad][:5]} " \
                              f"vs {a[bad][:5]}, margins {mg[bad][:5]}"
        e = np.abs(lp - logp)[~diff]
        assert np.all(e <= (2 * lb + 2e-5)[~diff]), e.max()
    else:
        excused = 0
        e = np.abs(a - action)
        assert np.all(e <= bound[:, 0] + 1e-5), (e.max(), np.argmax(e))
        st["action_err"] = max(st.get("action_err", 0.0), float(e.max(initial=0.0)))
        e = np.abs(lp - logp)
        assert np.all(e <= 1e-4), e.max()
    st["logp_err"] = max(st.get("logp_err", 0.0), float(e.max(initial=0.0)))
    st["excused_actions"] = st.get("excused_actions", 0) + excused
    st["decisions"] = st.get("decisions", 0) + (len(rows) if n_act else 0)
    return excused

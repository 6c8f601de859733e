"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds none of the roll-out arithmetic: it only draws the inputs
the method consumes (policy weights, the shared potential of the reaction
walk, agent counts of the market, trajectories for the returns pass) from
numpy's PCG64 generator and converts weights to their storage formats with
torch's own casts. The random numbers the method itself draws (actions,
resets, energy noise) come from Philox inside the kernels and the oracle.

Config shapes follow the paper's three example families (App. C): classic
control, a multi-agent economy and a noisy potential-energy walk; the
datasets and trained weights of the paper are not used.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import torch

CARTPOLE, PENDULUM, ACROBOT, MARKET, REACTION = 1, 2, 3, 4, 5

OBS_DIM = {CARTPOLE: 4, PENDULUM: 3, ACROBOT: 6, MARKET: 32, REACTION: 20}
STATE_DIM = {CARTPOLE: 4, PENDULUM: 2, ACROBOT: 4, MARKET: 32, REACTION: 21}
N_ACTIONS = {CARTPOLE: 2, PENDULUM: 0, ACROBOT: 0, MARKET: 50, REACTION: 40}
KIND_NAME = {CARTPOLE: "cartpole", PENDULUM: "pendulum", ACROBOT: "acrobot",
             MARKET: "market", REACTION: "reaction"}

# Layout of the reaction potential block (floats): A, centres, widths, amplitudes.
RX_DIM, RX_NG = 20, 64
RX_PARAM_FLOATS = RX_DIM * RX_DIM + RX_NG * RX_DIM + RX_NG + RX_NG


@dataclass
class Policy:
    """Policy weights in their storage format plus exact FP64 views.

    Layers are [out][in] row-major like torch.nn.Linear. The head has
    n_out + 1 rows; the last row is the value head.
    dtype 'f32': w* float32. 'bf16': w* uint16 bit patterns.
    'fp8': w* uint8 OCP E4M3FN codes with per-output-row float32 scales s*
    (powers of two), real weight = s[j] * fp8(code[j][k]); act_scale holds
    the power-of-two scale of each layer's input (observation, h1, h2).
    """

    dtype: str
    d_in: int
    h1: int
    h2: int
    n_head: int
    w1: np.ndarray
    w2: np.ndarray
    w3: np.ndarray
    b1: np.ndarray
    b2: np.ndarray
    b3: np.ndarray
    s1: np.ndarray
    s2: np.ndarray
    s3: np.ndarray
    log_std: np.ndarray = field(default_factory=lambda: np.zeros(1, np.float32))
    act_scale: tuple = (1.0, 1.0, 1.0)

    def exact(self, name: str) -> np.ndarray:
        """Exact real values (float64) of a weight, bias or scale array."""
        a = getattr(self, name)
        if name.startswith("b") or name.startswith("s") or name == "log_std":
            return a.astype(np.float64)
        if self.dtype == "f32":
            return a.astype(np.float64)
        if self.dtype == "bf16":
            return (a.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        scale = getattr(self, "s" + name[1:]).astype(np.float64)[:, None]
        vals = torch.from_numpy(a.copy()).view(torch.float8_e4m3fn).to(torch.float64).numpy()
        return vals * scale


def _to_storage(w: np.ndarray, dtype: str):
    """float32 weights -> (storage array, per-row scales) via torch casts."""
    ones = np.ones(w.shape[0], np.float32)
    if dtype == "f32":
        return w.astype(np.float32), ones
    if dtype == "bf16":
        t = torch.from_numpy(w.astype(np.float32)).to(torch.bfloat16)
        return t.view(torch.int16).numpy().view(np.uint16).copy(), ones
    if dtype == "fp8":
        amax = np.abs(w).max(axis=1).astype(np.float64)
        k = np.ceil(np.log2(np.maximum(amax, 1e-30) / 448.0))
        scale = np.where(amax > 0, np.exp2(k), 1.0).astype(np.float32)
        t = torch.from_numpy((w / scale[:, None]).astype(np.float32)).to(torch.float8_e4m3fn)
        return t.view(torch.uint8).numpy().copy(), scale
    raise ValueError(dtype)


def make_policy(d_in: int, h1: int, h2: int, n_out: int, dtype: str, seed: int = 0,
                std: float = 0.1, log_std_init: float = -0.5) -> Policy:
    """Weights and biases ~ N(0, std), converted to the storage dtype."""
    rng = np.random.default_rng(seed)
    n_head = n_out + 1
    w1 = rng.normal(0.0, std, (h1, d_in)).astype(np.float32)
    w2 = rng.normal(0.0, std, (h2, h1)).astype(np.float32)
    w3 = rng.normal(0.0, std, (n_head, h2)).astype(np.float32)
    b1 = rng.normal(0.0, std, h1).astype(np.float32)
    b2 = rng.normal(0.0, std, h2).astype(np.float32)
    b3 = rng.normal(0.0, std, n_head).astype(np.float32)
    q1, s1 = _to_storage(w1, dtype)
    q2, s2 = _to_storage(w2, dtype)
    q3, s3 = _to_storage(w3, dtype)
    # FP8 activation scales: observations up to 28 in magnitude, tanh outputs
    # (|h| < 1) mapped below 256; BF16 and FP32 inputs are not scaled.
    act_scale = (2.0 ** -4, 2.0 ** -8, 2.0 ** -8) if dtype == "fp8" else (1.0, 1.0, 1.0)
    return Policy(dtype, d_in, h1, h2, n_head, q1, q2, q3, b1, b2, b3, s1, s2, s3,
                  np.full(max(n_out, 1), log_std_init, np.float32), act_scale)


def policy_for(kind: int, dtype: str, h: int, seed: int = 0) -> Policy:
    n_act = N_ACTIONS[kind]
    return make_policy(OBS_DIM[kind], h, h, n_act if n_act else 1, dtype, seed)


def reaction_params(seed: int = 0) -> np.ndarray:
    """The shared 20-D potential as one float32 block.

    A = Q diag(lam) Q^T with lam ~ U[0.1, 2] and Q the sign-fixed QR factor of
    a 20x20 N(0,1) matrix; 64 centres ~ U[-3,3]^20, widths ~ U[0.3,1],
    amplitudes ~ N(0,1).
    """
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(RX_DIM, RX_DIM))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    lam = rng.uniform(0.1, 2.0, RX_DIM)
    A = (q * lam[None, :]) @ q.T
    A = 0.5 * (A + A.T)
    centres = rng.uniform(-3.0, 3.0, (RX_NG, RX_DIM))
    widths = rng.uniform(0.3, 1.0, RX_NG)
    amps = rng.normal(0.0, 1.0, RX_NG)
    return np.concatenate([A.ravel(), centres.ravel(), widths, amps]).astype(np.float32)


def agent_offsets(n_envs: int, lo: int = 5, hi: int = 100, seed: int = 0) -> np.ndarray:
    """CSR offsets [n_envs+1] of agent counts ~ U{lo..hi} (inclusive)."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(lo, hi + 1, n_envs)
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)


def trajectory(T: int, rows: int, p_done: float = 0.05, seed: int = 0):
    """Synthetic (reward, value, done, last_value) float32/uint8 arrays."""
    rng = np.random.default_rng(seed)
    reward = rng.normal(0.0, 1.0, (T, rows)).astype(np.float32)
    value = rng.normal(0.0, 1.0, (T, rows)).astype(np.float32)
    done = (rng.random((T, rows)) < p_done).astype(np.uint8)
    last_value = rng.normal(0.0, 1.0, rows).astype(np.float32)
    return reward, value, done, last_value


# The five workload configurations, by what they are.
CONFIGS = {
    "cartpole_1k": dict(kind=CARTPOLE, n_envs=1000, horizon=500, dtype="f32", hidden=64),
    "pendulum_10k": dict(kind=PENDULUM, n_envs=10000, horizon=200, dtype="bf16", hidden=256),
    "acrobot_10k": dict(kind=ACROBOT, n_envs=10000, horizon=200, dtype="bf16", hidden=256),
    "market_2k": dict(kind=MARKET, n_envs=2000, horizon=250, dtype="bf16", hidden=256),
    "reaction_4k": dict(kind=REACTION, n_envs=4096, horizon=1000, dtype="fp8", hidden=512),
}
GAMMA, LAMBDA = 0.99, 0.95

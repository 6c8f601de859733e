"""FP64 CPU oracle of the GPU-resident roll-out path (ctypes wrapper).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product
library never loads it and shares no code with it; both follow the same
written specification. The C source (``oracle.c``) is the oracle proper;
this module only marshals numpy arrays.

Paper anchors (arXiv 2408.00930): Sec. 2 and App. B (independent replicas
stepping in place, per-agent action sampling, in-place roll-out data), Sec. 3
(actor-critic for discrete and continuous actions), App. C (classic control,
multi-agent economics, noisy potential-energy walk).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CARTPOLE, PENDULUM, ACROBOT, MARKET, REACTION = 1, 2, 3, 4, 5
ACTION, RESET, ENV_NOISE = 0, 1, 2
F32, BF16, FP8 = 0, 1, 2
DTYPE_CODE = {"f32": F32, "bf16": BF16, "fp8": FP8}


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no -ffast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC",
             "-shared", "-Wall", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
        _declare(_lib)
    return _lib


class _Mlp(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("d_in", C.c_int32), ("h1", C.c_int32),
                ("h2", C.c_int32), ("n_head", C.c_int32),
                ("W1", C.c_void_p), ("b1", C.c_void_p), ("W2", C.c_void_p),
                ("b2", C.c_void_p), ("W3", C.c_void_p), ("b3", C.c_void_p),
                ("act_scale", C.c_double * 3)]


class _Env(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_envs", C.c_int32),
                ("agent_offsets", C.c_void_p), ("params", C.c_void_p)]


class _Traj(C.Structure):
    _fields_ = [("obs", C.c_void_p), ("action", C.c_void_p), ("reward", C.c_void_p),
                ("done", C.c_void_p), ("value", C.c_void_p), ("logp", C.c_void_p),
                ("last_value", C.c_void_p), ("margin_action", C.c_void_p),
                ("margin_done", C.c_void_p)]


def _declare(L):
    u32p = C.POINTER(C.c_uint32)
    dp = C.POINTER(C.c_double)
    L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
    L.orc_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                           C.c_uint32, u32p]
    L.orc_u01.argtypes = [C.c_uint32]
    L.orc_u01.restype = C.c_double
    L.orc_box_muller.argtypes = [C.c_double, C.c_double, dp, dp]
    for name in ("orc_round_bf16", "orc_round_fp8e4m3", "orc_wrap_angle"):
        getattr(L, name).argtypes = [C.c_double]
        getattr(L, name).restype = C.c_double
    L.orc_mlp_forward.argtypes = [C.POINTER(_Mlp), dp, dp]
    L.orc_mlp_adopt.argtypes = [C.POINTER(_Mlp), C.c_int64, dp, dp, dp, dp, dp,
                                C.POINTER(C.c_int32), dp]
    L.orc_sample_categorical.argtypes = [dp, C.c_int, C.c_double, dp, dp]
    L.orc_sample_categorical.restype = C.c_int
    L.orc_sample_gaussian.argtypes = [dp, dp, dp, C.c_int, dp, dp]
    L.orc_sample_rows.argtypes = [C.c_int64, C.c_int, C.c_int, dp, dp, C.c_uint64, C.c_uint32,
                                  u32p, C.c_uint32, dp, dp, dp]
    for name in ("orc_state_dim", "orc_obs_dim", "orc_n_actions"):
        getattr(L, name).argtypes = [C.c_int]
        getattr(L, name).restype = C.c_int
    L.orc_cartpole_accel.argtypes = [dp, C.c_double, dp, dp]
    L.orc_pendulum_accel.argtypes = [C.c_double, C.c_double]
    L.orc_pendulum_accel.restype = C.c_double
    L.orc_acrobot_deriv.argtypes = [dp, C.c_double, dp]
    L.orc_market_decode.argtypes = [C.c_int, dp, dp]
    L.orc_market_step.argtypes = [C.c_int, dp, C.POINTER(C.c_int), dp, dp]
    L.orc_market_step.restype = C.c_double
    L.orc_reaction_energy.argtypes = [dp, dp]
    L.orc_reaction_energy.restype = C.c_double
    L.orc_n_rows.argtypes = [C.POINTER(_Env)]
    L.orc_n_rows.restype = C.c_int64
    L.orc_env_reset.argtypes = [C.POINTER(_Env), C.c_uint64, C.c_uint32, C.c_uint32, dp]
    L.orc_observe.argtypes = [C.c_int, dp, dp]
    L.orc_env_step_row.argtypes = [C.POINTER(_Env), C.c_uint64, C.c_uint32, C.c_uint32,
                                   C.c_uint32, dp, C.c_double, dp, dp,
                                   C.POINTER(C.c_int), dp]
    L.orc_env_step_row.restype = C.c_int
    L.orc_reset_row.argtypes = [C.POINTER(_Env), C.c_uint64, C.c_uint32, C.c_uint32,
                                C.c_uint32, dp]
    L.orc_rollout.argtypes = [C.POINTER(_Env), C.POINTER(_Mlp), dp, C.c_uint64, C.c_uint32,
                              C.c_uint32, C.c_int32, dp, C.POINTER(_Traj)]
    L.orc_rollout.restype = C.c_int
    L.orc_cartpole_rollout_f32.argtypes = [C.POINTER(_Mlp), C.c_int64, C.c_uint64, C.c_uint32,
                                           C.c_uint32, C.c_int32, dp, dp, dp]
    L.orc_cartpole_rollout_f32.restype = C.c_int
    for name in ("orc_returns_gae", "orc_gae_bruteforce"):
        getattr(L, name).argtypes = [C.c_int32, C.c_int64, dp, dp, C.c_void_p, dp,
                                     C.c_double, C.c_double, C.c_int32, dp, dp]
    L.orc_num_threads.restype = C.c_int
    L.orc_ac_grad.argtypes = [C.POINTER(_Mlp), C.c_int, dp, C.c_int64, dp, dp, dp, dp,
                              C.c_double, C.c_double, C.c_int, dp, dp, dp, dp, dp, dp, dp]
    L.orc_ac_grad.restype = C.c_int
    L.orc_adam.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_int32, C.c_double, C.c_double,
                           C.c_double, C.c_double]


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ctype=C.c_double):
    return a.ctypes.data_as(C.POINTER(ctype))


# ---------------------------------------------------------------- RNG ----

def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def draw(seed, t, row, purpose, sub, epoch):
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_draw(seed, t, row, purpose, sub, epoch, _ptr(out, C.c_uint32))
    return out


def u01(x):
    return lib().orc_u01(int(x))


def box_muller(u1, u2):
    a, b = C.c_double(), C.c_double()
    lib().orc_box_muller(u1, u2, C.byref(a), C.byref(b))
    return a.value, b.value


# ----------------------------------------------------------- rounding ----

def round_bf16(x):
    f = lib().orc_round_bf16
    return np.array([f(float(v)) for v in np.ravel(x)]).reshape(np.shape(x))


def round_fp8(x):
    f = lib().orc_round_fp8e4m3
    return np.array([f(float(v)) for v in np.ravel(x)]).reshape(np.shape(x))


def wrap_angle(th):
    return lib().orc_wrap_angle(float(th))


# ---------------------------------------------------------------- MLP ----

class _MlpHold:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, dtype, W1, b1, W2, b2, W3, b3, act_scale=(1.0, 1.0, 1.0)):
        self.arrs = [_f64(a) for a in (W1, b1, W2, b2, W3, b3)]
        W1, b1, W2, b2, W3, b3 = self.arrs
        self.s = _Mlp(DTYPE_CODE[dtype] if isinstance(dtype, str) else dtype,
                      W1.shape[1], W1.shape[0], W2.shape[0], W3.shape[0],
                      *[a.ctypes.data for a in self.arrs],
                      (C.c_double * 3)(*[float(v) for v in act_scale]))


def mlp_hold(policy):
    """Build the C view of a policy from its exact (dequantised) weights."""
    return _MlpHold(policy.dtype, policy.exact("w1"), policy.exact("b1"),
                    policy.exact("w2"), policy.exact("b2"), policy.exact("w3"),
                    policy.exact("b3"), policy.act_scale)


def mlp_forward(policy, obs):
    """Policy head outputs [n, n_head] for observations [n, d_in]."""
    h = mlp_hold(policy) if not isinstance(policy, _MlpHold) else policy
    obs = _f64(np.atleast_2d(obs))
    out = np.zeros((obs.shape[0], h.s.n_head))
    for i in range(obs.shape[0]):
        row = _f64(obs[i])
        res = np.zeros(h.s.n_head)
        lib().orc_mlp_forward(C.byref(h.s), _ptr(row), _ptr(res))
        out[i] = res
    return out


U32 = 2.0 ** -24


def fp32_sum_bound(n_terms, abs_sum):
    """gamma_n * S: the bound of an FP32 sum of n terms whose magnitudes add
    up to S, in any order (Higham, Sec. 3.1)."""
    g = n_terms * U32 / (1.0 - n_terms * U32)
    return g * np.asarray(abs_sum)


def mlp_adopt(policy, obs, codes1, codes2):
    """Evaluate the policy from a device run's hidden-layer codes.

    obs [n, d_in] (the device's FP32 observations), codes1 [n, h1] and
    codes2 [n, h2] (real values of its quantised hidden outputs). Returns a
    dict: head [n, n_head] (FP64 from codes2), head_bound [n, n_head] (the
    error bound of the device's FP32 head), flips [n, 2] (codes that differ
    from the oracle's rounding, per layer) and ratio [n, 2] (the largest
    distance to the deciding midpoint in units of the activation's error
    bound; <= 1 for a legitimate flip)."""
    h = mlp_hold(policy) if not isinstance(policy, _MlpHold) else policy
    s = h.s
    obs = _f64(np.atleast_2d(obs))
    n = obs.shape[0]
    c1, c2 = _f64(codes1).reshape(n, s.h1), _f64(codes2).reshape(n, s.h2)
    out = {"head": np.zeros((n, s.n_head)), "head_bound": np.zeros((n, s.n_head)),
           "flips": np.zeros((n, 2), np.int32), "ratio": np.zeros((n, 2))}
    lib().orc_mlp_adopt(C.byref(s), n, _ptr(obs), _ptr(c1), _ptr(c2), _ptr(out["head"]),
                        _ptr(out["head_bound"]), _ptr(out["flips"], C.c_int32),
                        _ptr(out["ratio"]))
    return out


def sample_categorical(logits, u):
    lg = _f64(logits)
    lp, mg = C.c_double(), C.c_double()
    a = lib().orc_sample_categorical(_ptr(lg), lg.size, float(u), C.byref(lp), C.byref(mg))
    return a, lp.value, mg.value


def sample_rows(head, n_act, log_std, seed, t, rows, epoch):
    """Draws of the given rows at step t from their heads [n, n_head]:
    (action, logp, margin) arrays, margin = distance to the nearest CDF
    boundary (inf for Gaussian heads)."""
    h = _f64(np.atleast_2d(head))
    n, nh = h.shape
    r = np.ascontiguousarray(rows, dtype=np.uint32)
    ls = _f64(log_std if log_std is not None else np.zeros(1))
    a, lp, mg = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_sample_rows(n, nh, int(n_act), _ptr(h), _ptr(ls), seed, t,
                          _ptr(r, C.c_uint32), epoch, _ptr(a), _ptr(lp), _ptr(mg))
    return a, lp, mg


def sample_gaussian(mu, log_std, z):
    mu, ls, z = _f64(mu), _f64(log_std), _f64(z)
    a = np.zeros(mu.size)
    lp = C.c_double()
    lib().orc_sample_gaussian(_ptr(mu), _ptr(ls), _ptr(z), mu.size, _ptr(a), C.byref(lp))
    return a, lp.value


# --------------------------------------------------------------- envs ----

def state_dim(kind):
    return lib().orc_state_dim(kind)


def obs_dim(kind):
    return lib().orc_obs_dim(kind)


def n_actions(kind):
    return lib().orc_n_actions(kind)


def cartpole_accel(state, force):
    s = _f64(state)
    xdd, thdd = C.c_double(), C.c_double()
    lib().orc_cartpole_accel(_ptr(s), float(force), C.byref(xdd), C.byref(thdd))
    return xdd.value, thdd.value


def pendulum_accel(th, u):
    return lib().orc_pendulum_accel(float(th), float(u))


def acrobot_deriv(state, tau):
    s = _f64(state)
    out = np.zeros(4)
    lib().orc_acrobot_deriv(_ptr(s), float(tau), _ptr(out))
    return out


def market_decode(a):
    l, t = C.c_double(), C.c_double()
    lib().orc_market_decode(int(a), C.byref(l), C.byref(t))
    return l.value, t.value


def market_step(states, actions):
    s = _f64(states)
    n = s.shape[0]
    acts = np.ascontiguousarray(actions, dtype=np.int32)
    nxt = np.zeros_like(s)
    rew = np.zeros(n)
    price = lib().orc_market_step(n, _ptr(s), _ptr(acts, C.c_int), _ptr(nxt), _ptr(rew))
    return nxt, rew, price


def reaction_energy(params, x):
    p, xx = _f64(params), _f64(x)
    return lib().orc_reaction_energy(_ptr(p), _ptr(xx))


def observe(kind, state):
    s = _f64(state)
    out = np.zeros(obs_dim(kind))
    lib().orc_observe(kind, _ptr(s), _ptr(out))
    return out


class _EnvHold:
    def __init__(self, kind, n_envs, agent_offsets=None, params=None):
        self.kind = kind
        self.offsets = None if agent_offsets is None else np.ascontiguousarray(
            agent_offsets, dtype=np.int32)
        self.params = None if params is None else _f64(params)
        self.s = _Env(kind, n_envs,
                      None if self.offsets is None else self.offsets.ctypes.data,
                      None if self.params is None else self.params.ctypes.data)
        self.rows = int(lib().orc_n_rows(C.byref(self.s)))


def env_hold(kind, n_envs, agent_offsets=None, params=None):
    return _EnvHold(kind, n_envs, agent_offsets, params)


def env_reset(env, seed, epoch=0, t=0):
    """Reset every row at step t; returns states [rows, state_dim]."""
    st = np.zeros((env.rows, state_dim(env.kind)))
    lib().orc_env_reset(C.byref(env.s), seed, epoch, t, _ptr(st))
    return st


def env_step_row(env, state, action, seed=0, epoch=0, t=0, row=0):
    """One single-agent transition without auto-reset.

    Returns (next_state, reward, done, done_margin)."""
    s = _f64(state)
    nxt = np.zeros(state_dim(env.kind))
    rew, mg = C.c_double(), C.c_double()
    done = C.c_int()
    rc = lib().orc_env_step_row(C.byref(env.s), seed, epoch, t, row, _ptr(s), float(action),
                                _ptr(nxt), C.byref(rew), C.byref(done), C.byref(mg))
    if rc != 0:
        raise ValueError("no single-row transition for this environment kind")
    return nxt, rew.value, bool(done.value), mg.value


def reset_row(env, seed, epoch, t, row):
    st = np.zeros(state_dim(env.kind))
    lib().orc_reset_row(C.byref(env.s), seed, epoch, t, row, _ptr(st))
    return st


def rollout(env, policy, seed, epoch, t0, T, states, log_std=None, margins=True):
    """Free-running roll-out of T steps from `states` (copied, not modified).

    Returns a dict with obs [T,rows,obs_dim], action, reward, done, value, logp
    [T,rows], last_value [rows], margin_action, margin_done [T,rows] and the
    final states [rows, state_dim].
    """
    h = mlp_hold(policy) if not isinstance(policy, _MlpHold) else policy
    rows = env.rows
    od = obs_dim(env.kind)
    st = _f64(states).copy()
    out = {
        "obs": np.zeros((T, rows, od)), "action": np.zeros((T, rows)),
        "reward": np.zeros((T, rows)), "done": np.zeros((T, rows), dtype=np.uint8),
        "value": np.zeros((T, rows)), "logp": np.zeros((T, rows)),
        "last_value": np.zeros(rows),
        "margin_action": np.zeros((T, rows)) if margins else None,
        "margin_done": np.zeros((T, rows)) if margins else None,
    }
    tr = _Traj(*[None if out[k] is None else out[k].ctypes.data
                 for k in ("obs", "action", "reward", "done", "value", "logp",
                           "last_value", "margin_action", "margin_done")])
    ls = _f64(log_std if log_std is not None else np.zeros(1))
    rc = lib().orc_rollout(C.byref(env.s), C.byref(h.s), _ptr(ls), seed, epoch, t0, T,
                           _ptr(st), C.byref(tr))
    if rc != 0:
        raise ValueError(f"orc_rollout rejected its arguments (code {rc})")
    out["states"] = st
    return out


def cartpole_rollout_f32(policy, seed, epoch, t0, T, states):
    """The CartPole roll-out computed in FP32 throughout (the divergence
    envelope beside the FP64 oracle): obs [T, n, 4] and action [T, n]."""
    h = mlp_hold(policy) if not isinstance(policy, _MlpHold) else policy
    st = _f64(states)
    n = st.shape[0]
    obs = np.zeros((T, n, 4))
    act = np.zeros((T, n))
    rc = lib().orc_cartpole_rollout_f32(C.byref(h.s), n, seed, epoch, t0, T, _ptr(st), _ptr(obs),
                                        _ptr(act))
    if rc != 0:
        raise ValueError("not a CartPole FP32 policy")
    return {"obs": obs, "action": act}


# ------------------------------------------------------------ returns ----

def _gae_call(fn, reward, value, done, last_value, gamma, lam, bootstrap):
    r, v, lv = _f64(reward), _f64(value), _f64(last_value)
    d = np.ascontiguousarray(done, dtype=np.uint8)
    T, rows = r.shape
    ret = np.zeros((T, rows))
    adv = np.zeros((T, rows))
    fn(T, rows, _ptr(r), _ptr(v), d.ctypes.data, _ptr(lv), float(gamma), float(lam),
       int(bootstrap), _ptr(ret), _ptr(adv))
    return ret, adv


def returns_gae(reward, value, done, last_value, gamma, lam, bootstrap=True):
    """Recursive FP64 returns and GAE; arrays are [T, rows]."""
    return _gae_call(lib().orc_returns_gae, reward, value, done, last_value, gamma, lam,
                     bootstrap)


def gae_bruteforce(reward, value, done, last_value, gamma, lam, bootstrap=True):
    """O(T^2) explicit sums of the same quantities (for tiny T)."""
    return _gae_call(lib().orc_gae_bruteforce, reward, value, done, last_value, gamma, lam,
                     bootstrap)


def num_threads():
    return lib().orc_num_threads()


def set_threads(n):
    """Threads of the OpenMP loops over independent environments."""
    lib().orc_set_threads(int(n))


# ------------------------------------------------------ actor-critic update ----

def ac_grad(policy, n_act, obs, action, adv, ret, value_coef=0.5, entropy_coef=0.0,
            quant_backward=True, log_std=None):
    """Gradients of the actor-critic loss over the samples (obs [n, d_in],
    action [n], advantage [n], return [n]) as a dict of FP64 arrays shaped like
    the weights: w1 [h1][d_in], b1, w2 [h2][h1], b2, w3 [n_head][h2], b3 and,
    for Gaussian policies (n_act == 0), log_std."""
    h = mlp_hold(policy) if not isinstance(policy, _MlpHold) else policy
    s = h.s
    obs = _f64(np.atleast_2d(obs))
    n = obs.shape[0]
    action, adv, ret = _f64(action).reshape(n), _f64(adv).reshape(n), _f64(ret).reshape(n)
    if log_std is None:
        log_std = policy.exact("log_std") if hasattr(policy, "exact") else np.zeros(1)
    ls = _f64(np.atleast_1d(log_std))
    out = {"w1": np.zeros((s.h1, s.d_in)), "b1": np.zeros(s.h1), "w2": np.zeros((s.h2, s.h1)),
           "b2": np.zeros(s.h2), "w3": np.zeros((s.n_head, s.h2)), "b3": np.zeros(s.n_head),
           "log_std": np.zeros(1)}
    rc = lib().orc_ac_grad(C.byref(s), int(n_act), _ptr(ls), n, _ptr(obs), _ptr(action),
                           _ptr(adv), _ptr(ret), float(value_coef), float(entropy_coef),
                           1 if quant_backward else 0,
                           *[_ptr(out[k]) for k in ("w1", "b1", "w2", "b2", "w3", "b3",
                                                    "log_std")])
    if rc != 0:
        raise ValueError("actor-critic gradient not defined for this policy format")
    if n_act:
        del out["log_std"]
    return out


def adam(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on FP64 arrays (theta, m, v updated)."""
    for a in (theta, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib().orc_adam(theta.size, _ptr(theta), _ptr(g), _ptr(m), _ptr(v), int(t), float(lr),
                   float(b1), float(b2), float(eps))

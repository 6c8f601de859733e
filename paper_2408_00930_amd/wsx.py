"""Thin ctypes binding of libwsx.so (include/wsx.h), argument marshalling only.

torch provides the device memory (tensors) and the stream (torch's current
stream); every step of the roll-out runs in the library's HIP kernels. torch
is imported before the library is loaded so that the library binds to the HIP
runtime torch has already loaded. There is no fallback: if the library is
missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwsx.so")

CARTPOLE, PENDULUM, ACROBOT, MARKET, REACTION = 1, 2, 3, 4, 5
F32, BF16, FP8_E4M3, F64 = 0, 1, 2, 3
MODE_FUSED, MODE_PLAIN, MODE_GRAPH, MODE_FUSED_GRAPH = 0, 1, 2, 3
DTYPE_CODE = {"f32": F32, "bf16": BF16, "fp8": FP8_E4M3}

OBS_DIM = {CARTPOLE: 4, PENDULUM: 3, ACROBOT: 6, MARKET: 32, REACTION: 20}
STATE_DIM = {CARTPOLE: 4, PENDULUM: 2, ACROBOT: 4, MARKET: 32, REACTION: 21}
N_ACTIONS = {CARTPOLE: 2, PENDULUM: 0, ACROBOT: 0, MARKET: 50, REACTION: 40}


class WsxError(RuntimeError):
    pass


class _Policy(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("d_in", C.c_int32), ("h1", C.c_int32),
                ("h2", C.c_int32), ("n_head", C.c_int32),
                ("w1", C.c_void_p), ("w2", C.c_void_p), ("w3", C.c_void_p),
                ("b1", C.c_void_p), ("b2", C.c_void_p), ("b3", C.c_void_p),
                ("s1", C.c_void_p), ("s2", C.c_void_p), ("s3", C.c_void_p),
                ("act_scale", C.c_float * 3), ("log_std", C.c_void_p)]


class _Traj(C.Structure):
    _fields_ = [("capacity", C.c_int32), ("obs", C.c_void_p), ("action", C.c_void_p),
                ("reward", C.c_void_p), ("done", C.c_void_p), ("value", C.c_void_p),
                ("logp", C.c_void_p), ("last_value", C.c_void_p)]


class _EnvDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("tile_rows", C.c_int32), ("waves", C.c_int32),
                ("occupancy", C.c_int32), ("n_envs", C.c_int64),
                ("seed", C.c_uint64), ("state", C.c_void_p), ("agent_offsets", C.c_void_p),
                ("params", C.c_void_p)]


EXPORTS = ["wsx_env_state_bytes", "wsx_env_create", "wsx_env_reset", "wsx_rollout",
           "wsx_rollout_batch", "wsx_rollout_batch_ext",
           "wsx_env_info", "wsx_env_tiles", "wsx_env_set_step", "wsx_env_set_chunk",
           "wsx_env_destroy",
           "wsx_compute_returns",
           "wsx_policy_forward", "wsx_policy_trace", "wsx_quantize", "wsx_last_error"]

_lib = None


def lib():
    """Load libwsx.so (raises if it is missing: there is no other path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise WsxError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2408_00930_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32, u64, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_double
        L.wsx_env_state_bytes.argtypes = [i32, i64, i64, C.POINTER(C.c_size_t)]
        L.wsx_env_create.argtypes = [C.POINTER(_EnvDesc), C.POINTER(vp)]
        L.wsx_env_reset.argtypes = [vp, u32, vp]
        L.wsx_rollout.argtypes = [vp, C.POINTER(_Policy), i32, C.POINTER(_Traj), i32, vp]
        L.wsx_env_info.argtypes = [vp, C.POINTER(i64), C.POINTER(u32), C.POINTER(u32)]
        L.wsx_env_tiles.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
        L.wsx_env_set_step.argtypes = [vp, u32]
        L.wsx_env_set_chunk.argtypes = [vp, i32]
        L.wsx_env_destroy.argtypes = [vp]
        L.wsx_compute_returns.argtypes = [vp, vp, vp, vp, i32, i64, f64, f64, i32, vp, vp, i32, vp]
        L.wsx_policy_forward.argtypes = [C.POINTER(_Policy), vp, i64, vp, vp]
        L.wsx_policy_trace.argtypes = [vp, C.POINTER(_Policy), vp, i64, vp, vp, vp, vp]
        L.wsx_quantize.argtypes = [i32, C.c_float, vp, vp, i64, vp]
        L.wsx_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        raise WsxError(f"wsx error {rc}: {lib().wsx_last_error().decode()}")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ------------------------------------------------------------- policies ----

class DevicePolicy:
    """A policy's weights as device tensors plus the wsx_policy view of them."""

    def __init__(self, policy, device="cuda"):
        self.host = policy
        dev = torch.device(device)

        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        self.tensors = {n: t(getattr(policy, n)) for n in
                        ("w1", "w2", "w3", "b1", "b2", "b3", "s1", "s2", "s3", "log_std")}
        fp8 = policy.dtype == "fp8"
        g = self.tensors
        self.c = _Policy(DTYPE_CODE[policy.dtype], policy.d_in, policy.h1, policy.h2,
                         policy.n_head, g["w1"].data_ptr(), g["w2"].data_ptr(),
                         g["w3"].data_ptr(), g["b1"].data_ptr(), g["b2"].data_ptr(),
                         g["b3"].data_ptr(),
                         g["s1"].data_ptr() if fp8 else None,
                         g["s2"].data_ptr() if fp8 else None,
                         g["s3"].data_ptr() if fp8 else None,
                         (C.c_float * 3)(*policy.act_scale), g["log_std"].data_ptr())


# ----------------------------------------------------------- trajectory ----

class Trajectory:
    """Device trajectory buffers, [T][rows] (obs [T][rows][obs_dim])."""

    def __init__(self, kind, horizon, rows, device="cuda"):
        dev = torch.device(device)
        self.capacity = horizon
        self.obs = torch.empty((horizon, rows, OBS_DIM[kind]), dtype=torch.float32, device=dev)
        adt = torch.uint8 if N_ACTIONS[kind] else torch.float32
        self.action = torch.empty((horizon, rows), dtype=adt, device=dev)
        self.reward = torch.empty((horizon, rows), dtype=torch.float32, device=dev)
        self.done = torch.empty((horizon, rows), dtype=torch.uint8, device=dev)
        self.value = torch.empty((horizon, rows), dtype=torch.float32, device=dev)
        self.logp = torch.empty((horizon, rows), dtype=torch.float32, device=dev)
        self.last_value = torch.empty((rows,), dtype=torch.float32, device=dev)
        self.c = _Traj(horizon, *[_ptr(x) for x in (self.obs, self.action, self.reward,
                                                     self.done, self.value, self.logp,
                                                     self.last_value)])

    def host(self):
        return {k: getattr(self, k).cpu().numpy() for k in
                ("obs", "action", "reward", "done", "value", "logp", "last_value")}


# ----------------------------------------------------------------- envs ----

def env_state_bytes(kind, n_envs, n_rows):
    out = C.c_size_t()
    _check(lib().wsx_env_state_bytes(kind, n_envs, n_rows, C.byref(out)))
    return out.value


class Env:
    """An environment set: its device state block and the library handle."""

    def __init__(self, kind, n_envs, seed=0, agent_offsets=None, params=None, tile_rows=0,
                 waves=0, occupancy=0, device="cuda"):
        self.kind = kind
        self.n_envs = n_envs
        dev = torch.device(device)
        self.offsets = None if agent_offsets is None else np.ascontiguousarray(agent_offsets, np.int32)
        rows = int(self.offsets[-1]) if self.offsets is not None else n_envs
        self.rows = rows
        nbytes = env_state_bytes(kind, n_envs, rows)
        self.block = torch.zeros(nbytes, dtype=torch.uint8, device=dev)
        self.params = None if params is None else torch.from_numpy(
            np.ascontiguousarray(params, np.float32)).to(dev)
        desc = _EnvDesc(kind, tile_rows, waves, occupancy, n_envs, seed, self.block.data_ptr(),
                        None if self.offsets is None else self.offsets.ctypes.data,
                        None if self.params is None else self.params.data_ptr())
        h = C.c_void_p()
        _check(lib().wsx_env_create(C.byref(desc), C.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.wsx_env_destroy(self.handle)
            self.handle = None

    @property
    def state(self):
        """The state as a [state_dim, rows] float32 view (structure of arrays)."""
        sd = STATE_DIM[self.kind]
        return self.block[: sd * self.rows * 4].view(torch.float32).view(sd, self.rows)

    def tiles(self):
        """(tiles of the fused launch, rows one tile holds)."""
        n, cap = C.c_int32(), C.c_int32()
        _check(lib().wsx_env_tiles(self.handle, C.byref(n), C.byref(cap)))
        return n.value, cap.value

    def info(self):
        rows, step, epoch = C.c_int64(), C.c_uint32(), C.c_uint32()
        _check(lib().wsx_env_info(self.handle, C.byref(rows), C.byref(step), C.byref(epoch)))
        return rows.value, step.value, epoch.value

    def set_step(self, step):
        _check(lib().wsx_env_set_step(self.handle, step))

    def set_chunk(self, chunk_steps):
        """Steps per fused launch in MODE_FUSED_GRAPH (0 = the whole horizon)."""
        _check(lib().wsx_env_set_chunk(self.handle, chunk_steps))


def env_reset(env, epoch=0, stream=None):
    _check(lib().wsx_env_reset(env.handle, epoch, _stream(stream)))


def rollout(env, policy, horizon, traj, mode=MODE_FUSED, stream=None):
    _check(lib().wsx_rollout(env.handle, C.byref(policy.c), horizon, C.byref(traj.c), mode,
                             _stream(stream)))


def rollout_batch(envs, policies, horizon, trajs, stream=None):
    """Roll several environment sets out in one fused launch."""
    n = len(envs)
    L = lib()
    if not getattr(L, "_batch_sigs", False):
        L.wsx_rollout_batch.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                        C.c_int32, C.c_void_p]
        L._batch_sigs = True
    e = (C.c_void_p * n)(*[x.handle.value for x in envs])
    p = (C.POINTER(_Policy) * n)(*[C.pointer(x.c) for x in policies])
    t = (C.POINTER(_Traj) * n)(*[C.pointer(x.c) for x in trajs])
    _check(L.wsx_rollout_batch(e, p, t, n, horizon, _stream(stream)))


class _RolloutExt(C.Structure):
    _fields_ = [("reset", C.c_int32), ("epoch", C.c_uint32), ("returns", C.c_int32),
                ("bootstrap", C.c_int32), ("out_dtype", C.c_int32), ("gamma", C.c_double),
                ("lam", C.c_double), ("ret", C.c_void_p), ("adv", C.c_void_p)]


def rollout_batch_ext(envs, policies, horizon, trajs, epoch=None, returns=None, advantages=None,
                      gamma=0.99, lam=0.95, bootstrap=True, stream=None):
    """One fused launch: reset (if epoch is not None), roll-out of every set,
    then returns/GAE into the [horizon, rows] tensors `returns[i]`,
    `advantages[i]` (if given; float32 or float64)."""
    n = len(envs)
    L = lib()
    if not getattr(L, "_batch_ext_sigs", False):
        L.wsx_rollout_batch_ext.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                            C.c_int32, C.POINTER(_RolloutExt), C.c_void_p]
        L._batch_ext_sigs = True
    e = (C.c_void_p * n)(*[x.handle.value for x in envs])
    p = (C.POINTER(_Policy) * n)(*[C.pointer(x.c) for x in policies])
    t = (C.POINTER(_Traj) * n)(*[C.pointer(x.c) for x in trajs])
    x = _RolloutExt()
    x.reset = 0 if epoch is None else 1
    x.epoch = 0 if epoch is None else int(epoch)
    keep = []
    if returns is not None:
        code = {torch.float64: F64, torch.float32: F32}.get(returns[0].dtype, -1)
        r = (C.c_void_p * n)(*[_ptr(a) for a in returns])
        a = (C.c_void_p * n)(*[_ptr(a) for a in advantages])
        keep += [r, a]
        x.returns, x.bootstrap, x.out_dtype = 1, int(bootstrap), code
        x.gamma, x.lam = gamma, lam
        x.ret = C.cast(r, C.c_void_p).value
        x.adv = C.cast(a, C.c_void_p).value
    _check(L.wsx_rollout_batch_ext(e, p, t, n, horizon, C.byref(x), _stream(stream)))


def compute_returns(traj, horizon, gamma, lam, bootstrap=True, out_dtype=torch.float64,
                    returns=None, advantages=None, stream=None):
    rows = traj.reward.shape[1]
    if returns is None:
        returns = torch.empty((horizon, rows), dtype=out_dtype, device=traj.reward.device)
    if advantages is None:
        advantages = torch.empty((horizon, rows), dtype=out_dtype, device=traj.reward.device)
    code = F64 if out_dtype == torch.float64 else F32
    _check(lib().wsx_compute_returns(_ptr(traj.reward), _ptr(traj.value), _ptr(traj.done),
                                     _ptr(traj.last_value), horizon, rows, gamma, lam,
                                     int(bootstrap), _ptr(returns), _ptr(advantages), code,
                                     _stream(stream)))
    return returns, advantages


def compute_returns_raw(reward, value, done, last_value, gamma, lam, bootstrap=True,
                        out_dtype=torch.float64, stream=None):
    """Returns/GAE of raw [T][rows] device tensors."""
    T, rows = reward.shape
    ret = torch.empty((T, rows), dtype=out_dtype, device=reward.device)
    adv = torch.empty((T, rows), dtype=out_dtype, device=reward.device)
    code = F64 if out_dtype == torch.float64 else F32
    _check(lib().wsx_compute_returns(_ptr(reward), _ptr(value), _ptr(done), _ptr(last_value),
                                     T, rows, gamma, lam, int(bootstrap), _ptr(ret), _ptr(adv),
                                     code, _stream(stream)))
    return ret, adv


def policy_forward(policy, obs, stream=None):
    rows = obs.shape[0]
    head = torch.empty((rows, policy.host.n_head), dtype=torch.float32, device=obs.device)
    _check(lib().wsx_policy_forward(C.byref(policy.c), _ptr(obs), rows, _ptr(head),
                                    _stream(stream)))
    return head


def policy_trace(env, policy, obs, stream=None):
    """Head outputs [rows, n_head] and the quantised hidden-layer outputs
    h1, h2 [rows, hidden] (their real values, float64 on the host) from the
    kernel of env's roll-out."""
    rows = obs.shape[0]
    p = policy.host
    head = torch.empty((rows, p.n_head), dtype=torch.float32, device=obs.device)
    cdt = {"f32": torch.float32, "bf16": torch.bfloat16, "fp8": torch.float8_e4m3fn}[p.dtype]
    a1 = torch.empty((rows, p.h1), dtype=cdt, device=obs.device)
    a2 = torch.empty((rows, p.h2), dtype=cdt, device=obs.device)
    _check(lib().wsx_policy_trace(env.handle, C.byref(policy.c), _ptr(obs), rows, _ptr(head),
                                  _ptr(a1), _ptr(a2), _stream(stream)))
    h1 = a1.float().cpu().numpy().astype(np.float64) * p.act_scale[1]
    h2 = a2.float().cpu().numpy().astype(np.float64) * p.act_scale[2]
    return head, h1, h2


def quantize(dtype, x, scale=1.0, stream=None):
    y = torch.empty_like(x)
    _check(lib().wsx_quantize(dtype, scale, _ptr(x), _ptr(y), x.numel(), _stream(stream)))
    return y


# ---------------------------------------------------------------- server ----

class _ServerDesc(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("chunk_steps", C.c_int32),
                ("max_batch", C.c_int32)]


class _Request(C.Structure):
    _fields_ = [("kind", C.c_int32), ("horizon", C.c_int32), ("n_envs", C.c_int64),
                ("seed", C.c_uint64), ("epoch", C.c_uint32), ("keep_session", C.c_int32),
                ("session", C.c_int64), ("policy", C.POINTER(_Policy)),
                ("agent_offsets", C.c_void_p), ("params", C.c_void_p),
                ("gamma", C.c_double), ("lam", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_int32), ("session", C.c_int64),
                ("n_rows", C.c_int64), ("traj", _Traj), ("returns", C.c_void_p),
                ("advantages", C.c_void_p), ("queue_ms", C.c_double), ("latency_ms", C.c_double)]


class _ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("launches", C.c_int64), ("env_steps", C.c_int64), ("arena_in_use", C.c_size_t),
                ("arena_peak", C.c_size_t), ("queued", C.c_int32), ("running", C.c_int32)]


EXPORTS += ["wsx_server_create", "wsx_server_submit", "wsx_server_wait", "wsx_server_release",
            "wsx_server_cancel", "wsx_server_inject_launch_failure",
            "wsx_server_close_session", "wsx_server_get_stats", "wsx_server_destroy"]


def _server_sigs(L):
    if getattr(L, "_server_sigs", False):
        return
    vp = C.c_void_p
    L.wsx_server_create.argtypes = [C.POINTER(_ServerDesc), C.POINTER(vp)]
    L.wsx_server_submit.argtypes = [vp, C.POINTER(_Request), C.POINTER(C.c_int64)]
    L.wsx_server_wait.argtypes = [vp, C.c_int64, C.c_int32, C.POINTER(_Result)]
    L.wsx_server_release.argtypes = [vp, C.c_int64]
    L.wsx_server_cancel.argtypes = [vp, C.c_int64]
    L.wsx_server_inject_launch_failure.argtypes = [vp, C.c_int64]
    L.wsx_server_close_session.argtypes = [vp, C.c_int64]
    L.wsx_server_get_stats.argtypes = [vp, C.POINTER(_ServerStats)]
    L.wsx_server_destroy.argtypes = [vp]
    L._server_sigs = True


class Server:
    """Continuous-batching roll-out server over a device arena (a uint8 tensor)."""

    def __init__(self, arena_bytes, chunk_steps=25, max_batch=64, device="cuda"):
        L = lib()
        _server_sigs(L)
        self.arena = torch.empty(arena_bytes, dtype=torch.uint8, device=torch.device(device))
        d = _ServerDesc(self.arena.data_ptr(), arena_bytes, chunk_steps, max_batch)
        h = C.c_void_p()
        _check(L.wsx_server_create(C.byref(d), C.byref(h)))
        self.handle = h
        self._keep = {}   # request id -> host objects the request points at

    def submit(self, kind, policy, horizon, n_envs=0, seed=0, epoch=0, session=0, keep=False,
               agent_offsets=None, params=None, gamma=0.99, lam=0.95):
        offs = None if agent_offsets is None else np.ascontiguousarray(agent_offsets, np.int32)
        q = _Request(kind, horizon, n_envs, seed, epoch, int(keep), session, C.pointer(policy.c),
                     None if offs is None else offs.ctypes.data,
                     None if params is None else params.data_ptr(), gamma, lam)
        rid = C.c_int64()
        _check(lib().wsx_server_submit(self.handle, C.byref(q), C.byref(rid)))
        self._keep[rid.value] = (offs, params, policy)
        return rid.value

    def wait(self, rid, timeout_ms=-1):
        r = _Result()
        rc = lib().wsx_server_wait(self.handle, rid, timeout_ms, C.byref(r))
        if rc != 0:
            raise WsxError(f"wsx error {rc}: {lib().wsx_last_error().decode()}")
        return r

    def view(self, result, kind):
        """torch views (inside the arena) of a completed request's outputs."""
        base = self.arena.data_ptr()
        rows = result.n_rows
        T = result.traj.capacity

        def v(ptr, dtype, shape):
            itemsize = torch.empty((), dtype=dtype).element_size()
            n = int(np.prod(shape))
            off = ptr - base
            return self.arena[off:off + n * itemsize].view(dtype).view(*shape)
        adt = torch.uint8 if N_ACTIONS[kind] else torch.float32
        t = result.traj
        return {"obs": v(t.obs, torch.float32, (T, rows, OBS_DIM[kind])),
                "action": v(t.action, adt, (T, rows)),
                "reward": v(t.reward, torch.float32, (T, rows)),
                "done": v(t.done, torch.uint8, (T, rows)),
                "value": v(t.value, torch.float32, (T, rows)),
                "logp": v(t.logp, torch.float32, (T, rows)),
                "last_value": v(t.last_value, torch.float32, (rows,)),
                "returns": v(result.returns, torch.float32, (T, rows)),
                "advantages": v(result.advantages, torch.float32, (T, rows))}

    def release(self, rid):
        _check(lib().wsx_server_release(self.handle, rid))
        self._keep.pop(rid, None)

    def close_session(self, sid):
        _check(lib().wsx_server_close_session(self.handle, sid))

    def cancel(self, rid):
        _check(lib().wsx_server_cancel(self.handle, rid))

    def inject_launch_failure(self, rid):
        """Test support: the request's next launch is reported as failed."""
        _check(lib().wsx_server_inject_launch_failure(self.handle, rid))

    def stats(self):
        s = _ServerStats()
        _check(lib().wsx_server_get_stats(self.handle, C.byref(s)))
        return {k: getattr(s, k) for k, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().wsx_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ autotuner ----

class _TuneEntry(C.Structure):
    _fields_ = [("tile_rows", C.c_int32), ("waves", C.c_int32), ("occupancy", C.c_int32),
                ("chunk_steps", C.c_int32), ("us_per_step", C.c_double)]


EXPORTS += ["wsx_autotune_workspace_bytes", "wsx_autotune", "wsx_tune_lookup", "wsx_tune_save",
            "wsx_tune_load", "wsx_env_shape", "wsx_autotune_batch_workspace_bytes",
            "wsx_autotune_batch"]


def _tune_sigs(L):
    if getattr(L, "_tune_sigs", False):
        return
    vp = C.c_void_p
    L.wsx_autotune_workspace_bytes.argtypes = [C.POINTER(_EnvDesc), C.c_int32,
                                               C.POINTER(C.c_size_t)]
    L.wsx_autotune.argtypes = [C.POINTER(_EnvDesc), C.POINTER(_Policy), C.c_int32, C.c_int32, vp,
                               C.c_size_t, C.POINTER(_TuneEntry), vp]
    L.wsx_tune_lookup.argtypes = [C.c_int32, C.c_int64, C.c_int64, C.c_int32,
                                  C.POINTER(_TuneEntry)]
    L.wsx_tune_save.argtypes = [C.c_char_p]
    L.wsx_tune_load.argtypes = [C.c_char_p]
    L.wsx_env_shape.argtypes = [vp] + [C.POINTER(C.c_int32)] * 4
    L.wsx_autotune_batch_workspace_bytes.argtypes = [vp, C.c_int32, C.c_int32,
                                                     C.POINTER(C.c_size_t)]
    L.wsx_autotune_batch.argtypes = [vp, vp, C.c_int32, C.c_int32, C.c_int32, vp, C.c_size_t,
                                     C.POINTER(_TuneEntry), vp]
    L._tune_sigs = True


def _entry(e):
    return {k: getattr(e, k) for k, _ in _TuneEntry._fields_}


def autotune(kind, n_envs, policy, horizon, reps=3, seed=0, agent_offsets=None, params=None,
             stream=None):
    """Time every compiled kernel shape (and the graph chunk length) for this
    environment set and record the fastest in the library's table, so that an
    Env created later with the default shape uses it. Returns the entry."""
    L = lib()
    _tune_sigs(L)
    offs = None if agent_offsets is None else np.ascontiguousarray(agent_offsets, np.int32)
    par = None if params is None else torch.from_numpy(
        np.ascontiguousarray(params, np.float32)).cuda()
    desc = _EnvDesc(kind, 0, 0, 0, n_envs, seed, None,
                    None if offs is None else offs.ctypes.data,
                    None if par is None else par.data_ptr())
    need = C.c_size_t()
    _check(L.wsx_autotune_workspace_bytes(C.byref(desc), horizon, C.byref(need)))
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    out = _TuneEntry()
    _check(L.wsx_autotune(C.byref(desc), C.byref(policy.c), horizon, reps, ws.data_ptr(),
                          need.value, C.byref(out), _stream(stream)))
    return _entry(out)


def autotune_batch(sets, horizon, reps=3, stream=None):
    """The autotuner for sets rolled out together by rollout_batch. `sets` is a
    list of dicts (kind, n_envs, policy, seed, agent_offsets, params)."""
    L = lib()
    _tune_sigs(L)
    keep, descs = [], []
    for d in sets:
        offs = d.get("agent_offsets")
        offs = None if offs is None else np.ascontiguousarray(offs, np.int32)
        par = d.get("params")
        par = None if par is None else torch.from_numpy(np.ascontiguousarray(par, np.float32)).cuda()
        keep += [offs, par]
        descs.append(_EnvDesc(d["kind"], 0, 0, 0, d["n_envs"], d.get("seed", 0), None,
                              None if offs is None else offs.ctypes.data,
                              None if par is None else par.data_ptr()))
    n = len(descs)
    dp = (C.POINTER(_EnvDesc) * n)(*[C.pointer(x) for x in descs])
    pp = (C.POINTER(_Policy) * n)(*[C.pointer(d["policy"].c) for d in sets])
    need = C.c_size_t()
    _check(L.wsx_autotune_batch_workspace_bytes(dp, n, horizon, C.byref(need)))
    ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    out = _TuneEntry()
    _check(L.wsx_autotune_batch(dp, pp, n, horizon, reps, ws.data_ptr(), need.value,
                                C.byref(out), _stream(stream)))
    return _entry(out)


def tune_lookup(kind, n_envs, n_rows, cus):
    L = lib()
    _tune_sigs(L)
    out = _TuneEntry()
    rc = L.wsx_tune_lookup(kind, n_envs, n_rows, cus, C.byref(out))
    return None if rc != 0 else _entry(out)


def tune_save(path):
    L = lib()
    _tune_sigs(L)
    _check(L.wsx_tune_save(os.fsencode(path)))


def tune_load(path):
    L = lib()
    _tune_sigs(L)
    _check(L.wsx_tune_load(os.fsencode(path)))


def env_shape(env):
    """(tile_rows, waves, occupancy, chunk_steps) the set runs with."""
    L = lib()
    _tune_sigs(L)
    v = [C.c_int32() for _ in range(4)]
    _check(L.wsx_env_shape(env.handle, *[C.byref(x) for x in v]))
    return tuple(x.value for x in v)


# ------------------------------------------------------ actor-critic update ----

class _Grads(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("w1", "b1", "w2", "b2", "w3", "b3", "log_std")]


EXPORTS += ["wsx_ac_grad_workspace_bytes", "wsx_ac_grad", "wsx_ac_grad_static", "wsx_adam_step",
            "wsx_adam_step_many"]


def _update_sigs(L):
    if getattr(L, "_update_sigs", False):
        return
    vp = C.c_void_p
    L.wsx_ac_grad_workspace_bytes.argtypes = [C.POINTER(_Policy), C.c_int64,
                                              C.POINTER(C.c_size_t)]
    L.wsx_ac_grad.argtypes = [C.POINTER(_Policy), C.c_int32, vp, vp, vp, vp, C.c_int64,
                              C.c_float, C.c_float, C.POINTER(_Grads), vp, C.c_size_t, vp]
    L.wsx_ac_grad_static.argtypes = [C.POINTER(_Policy), C.c_int32, vp, vp, vp, vp, C.c_int64,
                                     C.c_float, C.c_float, C.POINTER(_Grads), vp]
    L.wsx_adam_step.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int32, C.c_float, C.c_float,
                                C.c_float, C.c_float, vp, C.c_int32, vp]
    L.wsx_adam_step_many.argtypes = [C.POINTER(_AdamTensor), C.c_int32, C.c_int32, C.c_float,
                                     C.c_float, C.c_float, C.c_float, vp]
    L._update_sigs = True


class _AdamTensor(C.Structure):
    _fields_ = [("param", C.c_void_p), ("grad", C.c_void_p), ("m", C.c_void_p),
                ("v", C.c_void_p), ("n", C.c_int64), ("store", C.c_void_p),
                ("store_dtype", C.c_int32)]


class Grads:
    """FP32 gradient tensors shaped like a policy's weights (device)."""

    NAMES = ("w1", "b1", "w2", "b2", "w3", "b3", "log_std")

    def __init__(self, policy, device="cuda"):
        h = policy.host if isinstance(policy, DevicePolicy) else policy
        shapes = {"w1": (h.h1, h.d_in), "b1": (h.h1,), "w2": (h.h2, h.h1), "b2": (h.h2,),
                  "w3": (h.n_head, h.h2), "b3": (h.n_head,), "log_std": (1,)}
        self.tensors = {n: torch.zeros(shapes[n], dtype=torch.float32, device=device)
                        for n in self.NAMES}
        self.c = _Grads(*[self.tensors[n].data_ptr() for n in self.NAMES])

    def __getitem__(self, name):
        return self.tensors[name]


def ac_grad_workspace_bytes(policy, samples):
    L = lib()
    _update_sigs(L)
    need = C.c_size_t()
    _check(L.wsx_ac_grad_workspace_bytes(C.byref(policy.c), int(samples), C.byref(need)))
    return need.value


def ac_grad(policy, n_actions, obs, action, returns, advantages, value_coef=0.5,
            entropy_coef=0.0, grads=None, workspace=None, stream=None):
    """Gradient of the actor-critic loss over the samples (flat views of a
    trajectory's fields: obs [n][d_in], action [n], returns and advantages
    [n] float32, all on the device). n_actions: K for a categorical policy,
    0 for a Gaussian one. Returns a Grads."""
    L = lib()
    _update_sigs(L)
    n = int(returns.numel())
    for t in (obs, action, returns, advantages):
        assert t.is_cuda and t.is_contiguous()
    assert obs.numel() == n * policy.host.d_in and action.numel() == n and advantages.numel() == n
    need = C.c_size_t()
    _check(L.wsx_ac_grad_workspace_bytes(C.byref(policy.c), n, C.byref(need)))
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    grads = grads or Grads(policy)
    _check(L.wsx_ac_grad(C.byref(policy.c), int(n_actions), obs.data_ptr(), action.data_ptr(),
                         returns.data_ptr(), advantages.data_ptr(), n, float(value_coef),
                         float(entropy_coef), C.byref(grads.c), workspace.data_ptr(),
                         workspace.numel(), _stream(stream)))
    return grads


AC_STATIC_MAX_SAMPLES = 2048


def ac_grad_static(policy, n_actions, obs, action, returns, advantages, value_coef=0.5,
                   entropy_coef=0.0, grads=None, stream=None):
    """ac_grad through wsx_ac_grad_static: no workspace argument and no
    allocation in the library (at most AC_STATIC_MAX_SAMPLES samples)."""
    L = lib()
    _update_sigs(L)
    n = int(returns.numel())
    grads = grads or Grads(policy)
    _check(L.wsx_ac_grad_static(C.byref(policy.c), int(n_actions), obs.data_ptr(),
                                action.data_ptr(), returns.data_ptr(), advantages.data_ptr(), n,
                                float(value_coef), float(entropy_coef), C.byref(grads.c),
                                _stream(stream)))
    return grads


def adam_step(param, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, store=None,
              stream=None):
    """One Adam step on FP32 device tensors in place; `store` (optional) is a
    tensor of the same size in float32 or bfloat16 that receives the new
    values (a policy's own weight buffer)."""
    L = lib()
    _update_sigs(L)
    n = param.numel()
    for t in (param, grad, m, v):
        assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float32 and t.numel() == n
    sd = F32
    if store is not None:
        assert store.numel() == n and store.is_contiguous()
        sd = BF16 if store.dtype in (torch.bfloat16, torch.int16, torch.uint16) else F32
    _check(L.wsx_adam_step(param.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), n,
                           int(step), float(lr), float(beta1), float(beta2), float(eps),
                           None if store is None else store.data_ptr(), sd, _stream(stream)))


def adam_step_many(tensors, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    """The same Adam step on several tensors in one launch: `tensors` is a
    list of (param, grad, m, v, store) with store None or a tensor as in
    adam_step."""
    L = lib()
    _update_sigs(L)
    arr = (_AdamTensor * max(1, len(tensors)))()
    for i, (param, grad, m, v, store) in enumerate(tensors):
        n = param.numel()
        for t in (param, grad, m, v):
            assert t.is_cuda and t.is_contiguous() and t.dtype == torch.float32 and t.numel() == n
        sd = F32
        if store is not None:
            assert store.numel() == n and store.is_contiguous()
            sd = BF16 if store.dtype in (torch.bfloat16, torch.int16, torch.uint16) else F32
        arr[i] = _AdamTensor(param.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(), n,
                             None if store is None else store.data_ptr(), sd)
    _check(L.wsx_adam_step_many(arr, len(tensors), int(step), float(lr), float(beta1),
                                float(beta2), float(eps), _stream(stream)))


# ----------------------------------------------------------- user kinds ----

class _UserKindDesc(C.Structure):
    _fields_ = [("state_dim", C.c_int32), ("obs_dim", C.c_int32), ("n_actions", C.c_int32),
                ("dtype", C.c_int32), ("hidden", C.c_int32)]


EXPORTS += ["wsx_user_kind_register"]


def user_kind_register(source, state_dim, obs_dim, n_actions, dtype, hidden):
    """Compile a user environment (C++ source of `struct UserEnv`) into the
    fused roll-out and return its new kind; the kind's sizes are recorded so
    Env and Trajectory work with it."""
    L = lib()
    L.wsx_user_kind_register.argtypes = [C.POINTER(_UserKindDesc), C.c_char_p,
                                         C.POINTER(C.c_int32)]
    d = _UserKindDesc(state_dim, obs_dim, n_actions,
                      DTYPE_CODE[dtype] if isinstance(dtype, str) else dtype, hidden)
    k = C.c_int32()
    _check(L.wsx_user_kind_register(C.byref(d), source.encode(), C.byref(k)))
    OBS_DIM[k.value] = obs_dim
    STATE_DIM[k.value] = state_dim
    N_ACTIONS[k.value] = n_actions
    return k.value

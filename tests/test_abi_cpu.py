"""The C-ABI library loads, exports every declared entry point, and rejects
bad arguments on the host before touching a GPU (no compute calls here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wsx.h")


def _lib():
    from paper_2408_00930_amd import wsx
    if not os.path.exists(wsx.LIB_PATH):
        pytest.skip("libwsx.so not built (run __graft_entry__.build())")
    return wsx, wsx.lib()


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(wsx_\w+)\s*\(", text, re.M)))


def test_header_declares_the_entry_points():
    names = declared()
    for n in ("wsx_env_create", "wsx_env_reset", "wsx_rollout", "wsx_compute_returns",
              "wsx_env_state_bytes", "wsx_env_destroy", "wsx_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    wsx, L = _lib()
    for n in declared():
        assert hasattr(L, n), n
    assert sorted(wsx.EXPORTS) == declared()


def test_state_bytes_validation():
    wsx, L = _lib()
    out = C.c_size_t()
    assert L.wsx_env_state_bytes(99, 10, 10, C.byref(out)) == -1
    assert b"unknown environment kind" in L.wsx_last_error()
    assert L.wsx_env_state_bytes(wsx.PENDULUM, 0, 0, C.byref(out)) == -1
    assert L.wsx_env_state_bytes(wsx.PENDULUM, 10, 12, C.byref(out)) == -1
    assert L.wsx_env_state_bytes(wsx.PENDULUM, 10, 10, C.byref(out)) == 0
    # state SoA + obs scratch + head scratch + step counter, 256-byte aligned
    assert out.value == 256 + 256 + 256 + 256
    assert L.wsx_env_state_bytes(wsx.MARKET, 3, 300, C.byref(out)) == 0
    assert out.value >= 300 * (32 + 32 + 51) * 4


def test_create_validation_without_gpu():
    wsx, L = _lib()
    h = C.c_void_p()
    assert L.wsx_env_create(None, C.byref(h)) == -1
    d = wsx._EnvDesc(wsx.MARKET, 0, 0, 0, 3, 0, 1234, None, None)
    assert L.wsx_env_create(C.byref(d), C.byref(h)) == -1           # market needs offsets
    assert b"agent_offsets" in L.wsx_last_error()
    d = wsx._EnvDesc(wsx.REACTION, 0, 0, 0, 3, 0, 1234, None, None)
    assert L.wsx_env_create(C.byref(d), C.byref(h)) == -1           # reaction needs params
    d = wsx._EnvDesc(wsx.PENDULUM, 129, 0, 0, 3, 0, 1234, None, None)
    assert L.wsx_env_create(C.byref(d), C.byref(h)) == -2           # no kernel holds 129-row tiles
    d = wsx._EnvDesc(wsx.PENDULUM, 0, 0, -1, 3, 0, 1234, None, None)
    assert L.wsx_env_create(C.byref(d), C.byref(h)) == -1           # negative occupancy
    d = wsx._EnvDesc(wsx.PENDULUM, -16, 0, 0, 3, 0, 1234, None, None)
    assert L.wsx_env_create(C.byref(d), C.byref(h)) == -1           # negative tile rows
    d = wsx._EnvDesc(wsx.PENDULUM, 0, 0, 0, 3, 0, None, None, None)
    assert L.wsx_env_create(C.byref(d), C.byref(h)) == -1           # no state block


def test_rollout_and_returns_validation_without_gpu():
    wsx, L = _lib()
    assert L.wsx_rollout(None, None, 1, None, 0, None) == -1
    assert L.wsx_env_set_chunk(None, 4) == -1
    assert L.wsx_compute_returns(None, None, None, None, 10, 10, 1.5, 0.9, 1, None, None,
                                 wsx.F64, None) == -1
    assert L.wsx_compute_returns(None, None, None, None, 10, 10, 0.9, 0.9, 1, None, None,
                                 wsx.BF16, None) == -2
    assert L.wsx_compute_returns(None, None, None, None, 0, 10, 0.9, 0.9, 1, None, None,
                                 wsx.F64, None) == 0                 # empty: nothing to do
    assert L.wsx_quantize(wsx.FP8_E4M3, 0.3, None, None, 4, None) == -1
    assert b"power of two" in L.wsx_last_error()


def test_server_validation_without_gpu():
    wsx, L = _lib()
    wsx._server_sigs(L)
    h = C.c_void_p()
    d = wsx._ServerDesc(None, 0, 25, 64)
    assert L.wsx_server_create(C.byref(d), C.byref(h)) == -1
    d = wsx._ServerDesc(1234, 1 << 30, 0, 64)
    assert L.wsx_server_create(C.byref(d), C.byref(h)) == -1      # chunk_steps must be > 0
    d = wsx._ServerDesc(1234, 1024, 25, 64)
    assert L.wsx_server_create(C.byref(d), C.byref(h)) == -1      # smaller than launch tables
    assert L.wsx_server_submit(None, None, None) == -1


def test_tuning_table_round_trip_and_rejects_bad_files(tmp_path):
    wsx, L = _lib()
    wsx._tune_sigs(L)
    good = tmp_path / "tune.txt"
    good.write_text("# kind n_envs n_rows cus tile_rows waves occupancy chunk_steps us_per_step\n"
                    "2 10007 10007 256 40 8 2 0 6.5\n"
                    "3 10007 10007 256 80 8 2 50 7.25\n"
                    "2 10007 10007 256 48 8 2 0 6.0\n")      # replaces the first pendulum line
    wsx.tune_load(str(good))
    e = wsx.tune_lookup(wsx.PENDULUM, 10007, 10007, 256)
    assert e == {"tile_rows": 48, "waves": 8, "occupancy": 2, "chunk_steps": 0,
                 "us_per_step": 6.0}
    assert wsx.tune_lookup(wsx.ACROBOT, 10007, 10007, 256)["chunk_steps"] == 50
    assert wsx.tune_lookup(wsx.PENDULUM, 10007, 10007, 304) is None     # other device
    out = tmp_path / "saved.txt"
    wsx.tune_save(str(out))
    lines = [l.split() for l in out.read_text().splitlines() if not l.startswith("#")]
    assert ["2", "10007", "10007", "256", "48", "8", "2", "0", "6"] in lines
    # a kernel shape that is not compiled, a malformed line: the file is refused whole
    for bad in ("2 500 500 256 200 8 2 0 1.0\n", "2 500 500 256 48 8 2\n",
                "9 500 500 256 48 8 2 0 1.0\n", "2 500 500 256 48 8 2 -1 1.0\n"):
        p = tmp_path / "bad.txt"
        p.write_text("2 777 777 256 48 8 2 0 1.0\n" + bad)
        with pytest.raises(wsx.WsxError):
            wsx.tune_load(str(p))
        assert wsx.tune_lookup(wsx.PENDULUM, 777, 777, 256) is None
    with pytest.raises(wsx.WsxError):
        wsx.tune_load(str(tmp_path / "missing.txt"))


def test_autotune_validation_without_gpu():
    wsx, L = _lib()
    wsx._tune_sigs(L)
    n = C.c_size_t()
    d = wsx._EnvDesc(wsx.PENDULUM, 0, 0, 0, 1000, 0, None, None, None)
    assert L.wsx_autotune_workspace_bytes(C.byref(d), 50, C.byref(n)) == 0
    # state block + 50 steps x 1000 rows x (obs 12 + action 4 + reward 4 + done 1 + value 4 +
    # logp 4) bytes + last value, each part rounded up to 256 bytes
    assert 50 * 1000 * 29 + 1000 * 4 <= n.value <= 50 * 1000 * 29 + 1000 * 4 + 64 * 1024
    assert L.wsx_autotune_workspace_bytes(C.byref(d), 0, C.byref(n)) == -1
    assert L.wsx_autotune(C.byref(d), None, 50, 3, 1234, n.value, None, None) == -1
    pol = wsx._Policy()
    assert L.wsx_autotune(C.byref(d), C.byref(pol), 50, 0, 1234, n.value, None, None) == -1
    assert L.wsx_autotune(C.byref(d), C.byref(pol), 50, 3, 1234, 16, None, None) == -1
    assert L.wsx_env_shape(None, None, None, None, None) == -1


def _fake_policy(wsx, dtype, d_in, h, n_head, log_std=True):
    p = 0x1000   # never dereferenced: validation rejects before any launch
    return wsx._Policy(dtype, d_in, h, h, n_head, p, p, p, p, p, p, None, None, None,
                       (C.c_float * 3)(1.0, 1.0, 1.0), p if log_std else None)


def test_update_validation_without_gpu():
    wsx, L = _lib()
    wsx._update_sigs(L)
    out = C.c_size_t()
    pend = _fake_policy(wsx, wsx.BF16, 3, 256, 2)
    assert L.wsx_ac_grad_workspace_bytes(C.byref(pend), 0, C.byref(out)) == -1
    assert L.wsx_ac_grad_workspace_bytes(C.byref(pend), 1000, C.byref(out)) == 0
    assert out.value >= 2 * 1000 * 256 * 2                    # h1 and dz2 rows, BF16
    fp8 = _fake_policy(wsx, wsx.FP8_E4M3, 20, 512, 41)
    assert L.wsx_ac_grad_workspace_bytes(C.byref(fp8), 10, C.byref(out)) == -2
    wide = _fake_policy(wsx, wsx.BF16, 3, 512, 2)
    assert L.wsx_ac_grad_workspace_bytes(C.byref(wide), 10, C.byref(out)) == -2
    g = wsx._Grads(*([0x1000] * 7))
    p = 0x1000
    # n_actions must match the head: Gaussian needs n_head 2, categorical K + 1
    assert L.wsx_ac_grad(C.byref(pend), 3, p, p, p, p, 10, 0.5, 0.0, C.byref(g), p, 1 << 30,
                         None) == -1
    cart = _fake_policy(wsx, wsx.F32, 4, 64, 3, log_std=False)
    assert L.wsx_ac_grad(C.byref(cart), 0, p, p, p, p, 10, 0.5, 0.0, C.byref(g), p, 1 << 30,
                         None) == -2
    assert L.wsx_ac_grad(C.byref(pend), 0, p, p, p, p, 10, 0.5, 0.0, C.byref(g), p, 16,
                         None) == -1                            # workspace too small
    assert b"workspace" in L.wsx_last_error()
    assert L.wsx_ac_grad(C.byref(pend), 0, None, p, p, p, 10, 0.5, 0.0, C.byref(g), p, 1 << 30,
                         None) == -1
    assert L.wsx_ac_grad(C.byref(pend), 0, p, p, p, p, 10, float("nan"), 0.0, C.byref(g), p,
                         1 << 30, None) == -1
    # Adam
    assert L.wsx_adam_step(p, p, p, p, 10, 0, 1e-3, 0.9, 0.999, 1e-8, None, 0, None) == -1
    assert L.wsx_adam_step(p, p, p, p, 10, 1, 1e-3, 1.0, 0.999, 1e-8, None, 0, None) == -1
    assert L.wsx_adam_step(p, p, p, p, 10, 1, 1e-3, 0.9, 0.999, 1e-8, p, 2, None) == -1
    assert L.wsx_adam_step(None, None, None, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None, 0,
                           None) == 0
    # Adam on several tensors in one launch
    T = wsx._AdamTensor
    good = (T * 2)(T(p, p, p, p, 10, None, 0), T(p, p, p, p, 0, None, 0))
    assert L.wsx_adam_step_many(None, 1, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert L.wsx_adam_step_many(good, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert L.wsx_adam_step_many(good, 17, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert b"n_tensors" in L.wsx_last_error()
    assert L.wsx_adam_step_many(good, 2, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert L.wsx_adam_step_many(good, 2, 1, 1e-3, 0.9, 1.0, 1e-8, None) == -1
    bad = (T * 2)(T(p, p, p, p, 10, p, 2), T(p, p, p, p, 5, None, 0))
    assert L.wsx_adam_step_many(bad, 2, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert b"tensor 0" in L.wsx_last_error()
    null = (T * 2)(T(p, p, p, p, 10, None, 0), T(p, None, p, p, 5, None, 0))
    assert L.wsx_adam_step_many(null, 2, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    assert b"tensor 1" in L.wsx_last_error()
    neg = (T * 1)(T(p, p, p, p, -1, None, 0))
    assert L.wsx_adam_step_many(neg, 1, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -1
    empty = (T * 2)(T(None, None, None, None, 0, None, 0), T(None, None, None, None, 0, None, 0))
    assert L.wsx_adam_step_many(empty, 2, 1, 1e-3, 0.9, 0.999, 1e-8, None) == 0


def test_user_kind_validation_and_compile_errors_without_gpu():
    wsx, L = _lib()
    import user_envs
    with pytest.raises(wsx.WsxError, match="state_dim"):
        wsx.user_kind_register(user_envs.POINT_MASS, 0, 2, 0, "bf16", 256)
    with pytest.raises(wsx.WsxError, match="user kinds run"):
        wsx.user_kind_register(user_envs.POINT_MASS, 2, 2, 0, "fp8", 512)
    with pytest.raises(wsx.WsxError, match="does not compile"):
        wsx.user_kind_register("struct UserEnv { int x = ; };", 2, 2, 0, "bf16", 256)
    # sizes that disagree with the descriptor are a compile-time error too
    with pytest.raises(wsx.WsxError, match="sizes differ"):
        wsx.user_kind_register(user_envs.POINT_MASS, 3, 2, 0, "bf16", 256)
    # a valid source compiles here; loading needs a GPU
    with pytest.raises(wsx.WsxError, match="no HIP device"):
        wsx.user_kind_register(user_envs.POINT_MASS, 2, 2, 0, "bf16", 256)

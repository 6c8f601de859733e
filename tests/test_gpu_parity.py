"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (derivations in the design notes, "Tolerances"):
- dynamics, FP32 on the GPU: a state after one step within 2e-5 * max(1, |x|)
  of the oracle's step from the same state and action (Acrobot's RK4 with
  trigonometric terms: 1e-4); rewards likewise.
- policy outputs, every row: the trace kernel (the roll-out's own MLP code
  and shape) exposes the quantised hidden-layer codes; a code that differs
  from the oracle's FP64 rounding must lie within the FP32 error bound of the
  deciding midpoint (a counted flip), the oracle evaluates downstream from
  the device's codes, and the head must lie within its FP32 accumulation
  bound gamma_{K+16} sum|W3 h2| + u|y| (about 1e-5 to 2e-4 here).
- discrete actions: equal unless the oracle's draw lies within 2 max|logit
  error| + 1e-6 of a CDF boundary; every excused draw is counted.
- returns / GAE: FP64, relative 1e-12.
"""
import numpy as np
import pytest

import oracle as O
from gpu_cases import Case, check_policy_step, env_groups, say
from paper_2408_00930_amd import inputs

pytestmark = pytest.mark.gpu

GAMMA, LAM = inputs.GAMMA, inputs.LAMBDA


def _wsx():
    from paper_2408_00930_amd import wsx
    return wsx


# ------------------------------------------------------------ quantiser ----

def test_quantize_bf16_matches_oracle_rounding():
    import torch
    wsx = _wsx()
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-30, 2000),
                        rng.uniform(-3e38, 3e38, 2000)]).astype(np.float32)
    # exact bf16 midpoints (finite codes only; subnormal and normal)
    codes = rng.integers(0, 0x7F7F, 4000).astype(np.uint32)
    base = (codes << 16).view(np.float32)
    mids = ((codes << 16) | 0x8000).view(np.float32)
    x = np.concatenate([x, mids, base, -mids])
    say("quantize bf16", x.size)
    y = wsx.quantize(wsx.BF16, torch.from_numpy(x).cuda()).cpu().numpy().astype(np.float64)
    want = O.round_bf16(x.astype(np.float64))
    bad = np.nonzero(y != want)[0]
    for i in bad[:10]:
        print(f"bf16 mismatch x={x[i]!r} ({x[i].view(np.uint32):08x}) gpu={y[i]!r} oracle={want[i]!r}")
    assert len(bad) == 0


@pytest.mark.parametrize("scale", [1.0, 2.0 ** -4, 2.0 ** -8])
def test_quantize_fp8_matches_oracle_rounding(scale):
    import torch
    wsx = _wsx()
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(0, 100, 20000), rng.normal(0, 0.01, 5000),
                        rng.uniform(-600, 600, 2000)]) * scale
    vals = np.unique(np.abs(O.round_fp8(np.linspace(-448, 448, 5000))))
    mids = (vals[:-1] + vals[1:]) / 2 * scale
    x = np.concatenate([x, mids, -mids]).astype(np.float32)
    say("quantize fp8", scale, x.size)
    y = wsx.quantize(wsx.FP8_E4M3, torch.from_numpy(x).cuda(), scale).cpu().numpy()
    want = np.array([scale * O.round_fp8(v / scale) for v in x.astype(np.float64)])
    assert np.array_equal(y.astype(np.float64), want)


# --------------------------------------------------------------- policy ----

@pytest.mark.parametrize("kind", [O.CARTPOLE, O.PENDULUM, O.ACROBOT, O.MARKET, O.REACTION])
@pytest.mark.parametrize("rows", [1, 37, 200])
def test_policy_forward_matches_oracle(kind, rows):
    """Every row within the head's FP32 bound of the oracle evaluated from the
    device's hidden-layer codes; wsx_policy_forward equals the trace kernel of
    a set with the kind's default shape bit for bit."""
    import json
    import torch
    from gpu_cases import adopted_head, flip_stats
    wsx = _wsx()
    c = Case(kind, 3, seed=3)
    rng = np.random.default_rng(rows)
    obs = rng.normal(0, 1.0, (rows, c.policy.d_in)).astype(np.float32)
    say("policy_forward", kind, rows)
    head = wsx.policy_forward(c.dpol, torch.from_numpy(obs).cuda()).cpu().numpy()
    head_t, ad, bound, err = adopted_head(c.env, c.dpol, c.policy, obs)
    assert np.array_equal(head.astype(np.float64), head_t)
    st = {"kind": kind, "dtype": c.policy.dtype}
    flip_stats(ad, err, bound, st)
    print("PRECISION " + json.dumps(st), flush=True)


# -------------------------------------------------------------- returns ----

@pytest.mark.parametrize("T,rows", [(1, 1), (63, 31), (64, 33), (65, 32), (200, 100),
                                    (1000, 7), (129, 257),
                                    # row-parallel kernel (>= 24 rows per CU), including
                                    # horizons just past one and sixteen 16-step blocks
                                    (3, 10000), (70, 12001), (200, 10000), (33, 8000),
                                    (256, 6500), (257, 7000),
                                    # segmented kernel on few rows: up to sixteen
                                    # one-block segments, then segments of several
                                    # 32-step blocks past 512 steps
                                    (500, 1000), (512, 65), (513, 70), (300, 6200),
                                    (1000, 4096), (4000, 130)])
@pytest.mark.parametrize("boot", [True, False])
def test_returns_match_oracle(T, rows, boot):
    import torch
    wsx = _wsx()
    r, v, d, lv = inputs.trajectory(T, rows, p_done=0.05, seed=T + rows)
    dev = [torch.from_numpy(a).cuda() for a in (r, v, d, lv)]
    say("returns", T, rows, boot)
    g, a = wsx.compute_returns_raw(*dev, GAMMA, LAM, boot)
    g, a = g.cpu().numpy(), a.cpu().numpy()
    gw, aw = O.returns_gae(r, v, d, lv, GAMMA, LAM, boot)
    assert np.allclose(g, gw, rtol=1e-12, atol=1e-12)
    assert np.allclose(a, aw, rtol=1e-12, atol=1e-12)
    if boot and T >= 200:
        import json
        print("PRECISION " + json.dumps({"returns": [T, rows], "G_rel": float(_rel(g, gw).max()),
                                         "A_rel": float(_rel(a, aw).max())}), flush=True)
    # FP32 outputs: the FP64 result rounded once (a last-bit FP64 difference can
    # round the other way, so one FP32 ulp is allowed)
    g32, a32 = wsx.compute_returns_raw(*dev, GAMMA, LAM, boot, out_dtype=torch.float32)
    assert np.allclose(g32.cpu().numpy(), gw, rtol=1.2e-7, atol=1e-7)
    assert np.allclose(a32.cpu().numpy(), aw, rtol=1.2e-7, atol=1e-7)


@pytest.mark.parametrize("T", [8, 200, 250, 500, 1000])
@pytest.mark.parametrize("rows", [5, 10000])
def test_returns_geometric_closed_form(T, rows):
    import torch
    wsx = _wsx()
    r = torch.ones((T, rows), device="cuda")
    v = torch.zeros((T, rows), device="cuda")
    d = torch.zeros((T, rows), dtype=torch.uint8, device="cuda")
    lv = torch.zeros(rows, device="cuda")
    say("returns closed form", T)
    g, _ = wsx.compute_returns_raw(r, v, d, lv, 0.99, 0.95, False)
    assert np.allclose(g[0].cpu().numpy(), (1 - 0.99 ** T) / (1 - 0.99), rtol=1e-13, atol=0)


# ---------------------------------------------------------------- reset ----

@pytest.mark.parametrize("kind", [O.CARTPOLE, O.PENDULUM, O.ACROBOT, O.MARKET, O.REACTION])
def test_reset_matches_oracle(kind):
    wsx = _wsx()
    c = Case(kind, 50, seed=7)
    say("reset", kind)
    wsx.env_reset(c.env, epoch=3)
    got = c.gpu_state()
    want = O.env_reset(c.ohold, 7, 3, 0)
    tol = 2e-4 if kind == O.REACTION else 2e-6     # reaction: FP32 energy of the start
    assert np.allclose(got, want, rtol=1e-6, atol=tol)
    assert c.env.info()[1:] == (0, 3)


# ------------------------------------------------------------- lock-step ----

DYN_TOL = {O.CARTPOLE: 2e-5, O.PENDULUM: 2e-5, O.ACROBOT: 1e-4, O.MARKET: 2e-5,
           O.REACTION: 2e-4}


def _close(a, b, tol):
    return np.abs(a - b) <= tol * np.maximum(1.0, np.abs(b))


def _rel(a, b):
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


def lockstep(case, T, epoch=1, start=None, stats=None):
    """Step the GPU one step per call; validate each step against the oracle.

    Returns (n_decisions, n_excused); `stats` (a dict), if given, receives the
    largest errors seen per field."""
    wsx = _wsx()
    kind = case.kind
    traj = wsx.Trajectory(kind, 1, case.rows)
    wsx.env_reset(case.env, epoch)
    if start is not None:
        case.set_gpu_state(start)
    n_dec = n_exc = 0
    st = stats if stats is not None else {}

    def worst(key, v):
        st[key] = max(st.get(key, 0.0), float(np.max(v, initial=0.0)))
    for t in range(T):
        s = case.gpu_state()
        say("lockstep", kind, "step", t, "rows", case.rows)
        wsx.rollout(case.env, case.dpol, 1, traj, wsx.MODE_FUSED)
        g = traj.host()
        s_next = case.gpu_state()
        ref = O.rollout(case.ohold, case.mlp, case.seed, epoch, t, 1, s, case.log_std)
        # observation of the state the step started from
        assert np.allclose(g["obs"][0], ref["obs"][0], rtol=0, atol=2e-6)
        worst("obs_abs", np.abs(g["obs"][0] - ref["obs"][0]))
        # policy: every row against the oracle with the device's rounding
        # decisions adopted (flips counted); the plain FP64 evaluation's
        # distance is reported beside it
        exc = check_policy_step(case.env, case.dpol, case.policy, kind, g["obs"][0],
                                g["value"][0], g["action"][0], g["logp"][0], case.seed, epoch, t,
                                np.arange(case.rows), case.log_std, st)
        n_exc += exc
        if O.n_actions(kind):
            n_dec += case.rows
        worst("value_vs_fp64_forward", np.abs(g["value"][0] - ref["value"][0]))
        act_g = g["action"][0].astype(np.float64)
        # dynamics of the GPU's own action from the GPU's state
        tol = DYN_TOL[kind]
        if kind == O.MARKET:
            for (r0, r1) in env_groups(case):
                nxt, rew, _ = O.market_step(s[r0:r1], act_g[r0:r1].astype(np.int32))
                assert np.all(_close(s_next[r0:r1], nxt, tol))
                assert np.all(_close(g["reward"][0][r0:r1], rew, tol))
                worst("state_rel", _rel(s_next[r0:r1], nxt))
                worst("reward_rel", _rel(g["reward"][0][r0:r1], rew))
            assert not g["done"].any()
        else:
            for r in range(case.rows):
                nxt, rew, done, dm = O.env_step_row(case.ohold, s[r], act_g[r], case.seed, epoch,
                                                    t, r)
                if bool(g["done"][0][r]) != done:
                    assert dm < 1e-5, f"termination flip far from the threshold (row {r})"
                    n_exc += 1
                    continue
                if done:
                    nxt = O.reset_row(case.ohold, case.seed, epoch, t + 1, r)
                assert np.all(_close(s_next[r], nxt, tol)), (r, s_next[r], nxt)
                assert _close(g["reward"][0][r], rew, tol)
                worst("state_rel", _rel(s_next[r], nxt))
                worst("reward_rel", _rel(g["reward"][0][r], rew))
    return n_dec, n_exc


@pytest.mark.parametrize("kind,n_envs,T", [(O.CARTPOLE, 100, 60), (O.PENDULUM, 100, 40),
                                           (O.ACROBOT, 100, 30), (O.MARKET, 6, 12),
                                           (O.REACTION, 40, 20)])
def test_lockstep_matches_oracle(kind, n_envs, T):
    import json
    c = Case(kind, n_envs, seed=11)
    stats = {}
    n_dec, n_exc = lockstep(c, T, stats=stats)
    print(f"kind {kind}: {n_dec} decisions, {n_exc} excused", flush=True)
    stats.update(kind=kind, dtype=c.policy.dtype, rows=c.rows, steps=T, excused=n_exc,
                 decisions=n_dec)
    print("PRECISION " + json.dumps(stats), flush=True)


def test_lockstep_acrobot_terminations():
    """Links raised: episodes end and restart from the RESET draw."""
    from paper_2408_00930_amd import wsx
    c = Case(O.ACROBOT, 64, seed=5)
    wsx.env_reset(c.env, 1)
    st = c.gpu_state()
    st[:, 0] += np.pi
    lockstep(c, 25, epoch=1, start=st)


def test_free_running_cartpole_matches_oracle():
    """FP32 CartPole from the same reset, compared step by step until the
    first excused decision of each env (then the env is excused and
    counted)."""
    wsx = _wsx()
    c = Case(O.CARTPOLE, 200, seed=2)
    T = 300
    traj = wsx.Trajectory(O.CARTPOLE, T, c.rows)
    wsx.env_reset(c.env, 0)
    say("free-running cartpole", T)
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
    print(f"free-running: {diverged} of {c.rows} envs hit an excused decision", flush=True)
    assert diverged <= c.rows // 50


# --------------------------------------------------- forms and invariants ----

def _run(case, mode, T, epoch=0):
    wsx = _wsx()
    traj = wsx.Trajectory(case.kind, T, case.rows)
    wsx.env_reset(case.env, epoch)
    wsx.rollout(case.env, case.dpol, T, traj, mode)
    out = traj.host()
    out["state"] = case.gpu_state()
    return out


KINDS_SMALL = [(O.CARTPOLE, 70), (O.PENDULUM, 90), (O.ACROBOT, 90), (O.MARKET, 7),
               (O.REACTION, 50)]


@pytest.mark.parametrize("kind,n", KINDS_SMALL)
def test_plain_and_graph_equal_fused_bitwise(kind, n):
    wsx = _wsx()
    c = Case(kind, n, seed=4)
    say("fused vs plain vs graph", kind)
    f = _run(c, wsx.MODE_FUSED, 9)
    p = _run(c, wsx.MODE_PLAIN, 9)
    for k in f:
        assert np.array_equal(f[k], p[k]), k
    g1 = _run(c, wsx.MODE_GRAPH, 9)
    g2 = _run(c, wsx.MODE_GRAPH, 9)     # replay of the cached graph
    for k in f:
        assert np.array_equal(f[k], g1[k]), k
        assert np.array_equal(f[k], g2[k]), k


@pytest.mark.parametrize("kind,n", KINDS_SMALL)
@pytest.mark.parametrize("chunk", [0, 4, 9])
def test_fused_graph_chunks_equal_fused_bitwise(kind, n, chunk):
    """The horizon as chunked fused launches in one graph, replayed three times
    into the same buffers with eager work in between, equals one launch."""
    import torch
    wsx = _wsx()
    c = Case(kind, n, seed=8)
    say("fused graph chunks", kind, chunk)
    f = _run(c, wsx.MODE_FUSED, 9, epoch=3)
    c.env.set_chunk(chunk)
    traj = wsx.Trajectory(kind, 9, c.rows)
    for rep in range(3):
        wsx.env_reset(c.env, 3)
        wsx.rollout(c.env, c.dpol, 9, traj, wsx.MODE_FUSED_GRAPH)
        g = traj.host()
        g["state"] = c.gpu_state()
        for k in f:
            assert np.array_equal(f[k], g[k]), (rep, k)
        traj.reward.fill_(-7.0)            # eager work between the replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("kind,n", [(O.CARTPOLE, 70), (O.PENDULUM, 90), (O.MARKET, 7)])
@pytest.mark.parametrize("mode_name", ["MODE_GRAPH", "MODE_FUSED_GRAPH"])
def test_graph_replays_follow_the_reset_epoch(kind, n, mode_name):
    """A graph captured after a reset with one epoch and replayed into the same
    buffers after resets with other epochs draws from the new epoch's streams:
    every replay equals the fused launch of that epoch."""
    wsx = _wsx()
    c = Case(kind, n, seed=12)
    mode = getattr(wsx, mode_name)
    T = 7
    want = {e: _run(c, wsx.MODE_FUSED, T, epoch=e) for e in (1, 2, 5)}
    assert not np.array_equal(want[1]["obs"], want[2]["obs"])
    c.env.set_chunk(3)
    traj = wsx.Trajectory(kind, T, c.rows)
    for epoch in (1, 2, 5, 1):
        say("graph replay epoch", kind, mode_name, epoch)
        wsx.env_reset(c.env, epoch)
        wsx.rollout(c.env, c.dpol, T, traj, mode)
        g = traj.host()
        g["state"] = c.gpu_state()
        for k in want[epoch]:
            assert np.array_equal(want[epoch][k], g[k]), (epoch, k)


def test_fused_graph_horizon_zero_and_rejects_negative_chunk():
    wsx = _wsx()
    c = Case(O.PENDULUM, 40, seed=2)
    say("fused graph horizon 0")
    f = _run(c, wsx.MODE_FUSED, 0)
    c.env.set_chunk(5)
    g = _run(c, wsx.MODE_FUSED_GRAPH, 0)
    assert np.array_equal(f["last_value"], g["last_value"])
    with pytest.raises(wsx.WsxError):
        c.env.set_chunk(-1)


@pytest.mark.parametrize("kind,n", KINDS_SMALL)
def test_resume_split_is_bitwise(kind, n):
    wsx = _wsx()
    c = Case(kind, n, seed=6)
    say("resume split", kind)
    full = _run(c, wsx.MODE_FUSED, 12)
    wsx.env_reset(c.env, 0)
    t1 = wsx.Trajectory(kind, 5, c.rows)
    t2 = wsx.Trajectory(kind, 7, c.rows)
    wsx.rollout(c.env, c.dpol, 5, t1)
    a = t1.host()
    wsx.rollout(c.env, c.dpol, 7, t2)
    b = t2.host()
    for k in ("obs", "action", "reward", "done", "value", "logp"):
        assert np.array_equal(np.concatenate([a[k], b[k]]), full[k]), k
    assert np.array_equal(a["last_value"], full["value"][5])
    assert np.array_equal(b["last_value"], full["last_value"])
    assert c.env.info()[1] == 12


@pytest.mark.parametrize("kind,n", [(O.PENDULUM, 170), (O.MARKET, 9), (O.REACTION, 40)])
def test_replica_results_do_not_depend_on_other_replicas(kind, n):
    wsx = _wsx()
    big = Case(kind, n, seed=8)
    k = 3
    offsets = None if kind != O.MARKET else big.offsets[:k + 1]
    small = Case(kind, k, seed=8, offsets=offsets)
    say("replica independence", kind)
    fb = _run(big, wsx.MODE_FUSED, 6)
    fs = _run(small, wsx.MODE_FUSED, 6)
    rows = small.rows
    for key in ("obs", "action", "reward", "done", "value", "logp"):
        assert np.array_equal(fb[key][:, :rows], fs[key]), key


def test_horizon_zero_writes_only_last_value():
    wsx = _wsx()
    c = Case(O.PENDULUM, 33, seed=1)
    traj = wsx.Trajectory(O.PENDULUM, 1, c.rows)
    wsx.env_reset(c.env, 0)
    say("horizon 0")
    before = c.gpu_state()
    wsx.rollout(c.env, c.dpol, 0, traj)
    lv = traj.last_value.cpu().numpy()
    want = O.mlp_forward(c.policy, np.array([O.observe(O.PENDULUM, s) for s in before]))[:, -1]
    assert np.allclose(lv, want, atol=2e-2)
    assert np.array_equal(c.gpu_state(), before)


def test_market_extreme_env_sizes():
    """Envs of 1 agent and of a full tile (128 agents) next to ordinary ones."""
    counts = np.array([1, 128, 5, 100, 1, 64])
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    c = Case(O.MARKET, len(counts), seed=9, offsets=offsets)
    lockstep(c, 5)

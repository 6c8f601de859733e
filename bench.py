#!/usr/bin/env python3
"""Roll-out throughput on one MI355X: fused vs per-step-launch forms.

One step = the whole hot path over one batch: reset, roll-out over the
horizon and returns/GAE for every environment set of the workload. The
fused form runs all of it in one persistent launch (rollout_batch_ext); the
comparison forms run it as separate calls (fused_calls: reset and returns
kernels around the fused roll-out; plain / graph: per-step launches). The
default workload is 10,000 Pendulum + 10,000 Acrobot replicas, horizon 200,
BF16 policies obs-256-256-(1+1), both sets in the one launch, with the kernel
shape chosen by the library's autotuner. Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "env-steps/s fused vs per-step-launch at tolerance; p50/p99 rollout latency"
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}

# name -> list of (config key in inputs.CONFIGS)
# oracle sample of each workload's CPU baseline when it is a sub-record (about
# 1-5 s of the FP64 oracle on 16 host threads)
CPU_SAMPLE_ENVS = {"cartpole_1k": 1000, "market_2k": 32, "reaction_4k": 64,
                   "pendulum_acrobot_10k": 1024}

WORKLOADS = {
    "pendulum_acrobot_10k": ["pendulum_10k", "acrobot_10k"],
    "cartpole_1k": ["cartpole_1k"],
    "market_2k": ["market_2k"],
    "reaction_4k": ["reaction_4k"],
}


def policy_flops(pol):
    return 2 * (pol.d_in * pol.h1 + pol.h1 * pol.h2 + pol.h2 * pol.n_head)


def update_flops(pol):
    """Algorithmic FLOP of one sample of the actor-critic update: the forward
    pass again, then dz2 = dhead W3, dh1 = dz2 W2 and the weight gradients
    dW3, dW2, dW1 (unpadded MACs, two FLOP each)."""
    back = 2 * (2 * pol.n_head * pol.h2 + 2 * pol.h1 * pol.h2 + pol.h1 * pol.d_in)
    return policy_flops(pol) + back


def update_leg(sets, steps, wsx, torch):
    """The on-device actor-critic update over each set's last trajectory and
    returns: the gradient over every sample (wsx_ac_grad), then one Adam step
    per tensor into FP32 masters that write the policy's own weights. One
    untimed pass, then `steps` passes timed with events on the stream."""
    legs = []
    for s in sets:
        if s.policy.dtype not in ("f32", "bf16"):
            continue
        obs = s.traj.obs.reshape(-1, s.policy.d_in)
        act = s.traj.action.reshape(-1)
        r, a = s.ret.reshape(-1), s.adv.reshape(-1)
        g = wsx.Grads(s.dp)
        need = wsx.ac_grad_workspace_bytes(s.dp, r.numel())
        ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        names = ["w1", "b1", "w2", "b2", "w3", "b3"] + (["log_std"] if not wsx.N_ACTIONS[s.kind] else [])
        master = {k: torch.from_numpy(s.policy.exact(k).astype("float32")).cuda().reshape(-1)
                  for k in names}
        if "log_std" in master:
            master["log_std"] = master["log_std"][:1].clone()
        mom = {k: (torch.zeros_like(v), torch.zeros_like(v)) for k, v in master.items()}
        store = {k: s.dp.tensors[k].reshape(-1)[:master[k].numel()] for k in names}
        legs.append((s, obs, act, r, a, g, ws, names, master, mom, store))

    def one(t):
        items = []
        for s, obs, act, r, a, g, ws, names, master, mom, store in legs:
            wsx.ac_grad(s.dp, wsx.N_ACTIONS[s.kind], obs, act, r, a, 0.5, 0.01, grads=g,
                        workspace=ws)
            items += [(master[k], g[k].reshape(-1)[:master[k].numel()], mom[k][0], mom[k][1],
                       store[k]) for k in names]
        for i in range(0, len(items), 16):   # every tensor of the sets in one Adam launch
            wsx.adam_step_many(items[i:i + 16], t, 3e-4)
    if not legs:
        return None
    one(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for t in range(steps):
        one(t + 2)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    samples = sum(l[3].numel() for l in legs)
    flop = sum(update_flops(l[0].policy) * l[3].numel() for l in legs)
    dtype = legs[0][0].policy.dtype
    tflops = flop / (ms * 1e-3) / 1e12
    return {"samples": samples, "steps": steps, "ms_per_update": round(ms, 4),
            "samples_per_s": round(samples / ms * 1e3, 1),
            "flop_per_sample": {l[0].key: update_flops(l[0].policy) for l in legs},
            "achieved_tflops": round(tflops, 2), "peak_tflops": PEAK_TFLOPS[dtype],
            "frac": round(tflops / PEAK_TFLOPS[dtype], 4),
            "what": "gradient of the actor-critic loss over every sample of the sets' "
                    "trajectories plus one batched Adam launch over every policy tensor"}


def sweep(kind_key, counts, steps, wsx, inputs, torch):
    """Env-count sweep (the paper's throughput-vs-environments curves): for each
    count, the fused roll-out (autotuned shape) and the full training
    iteration (reset, roll-out, returns/GAE, gradient, Adam), one JSON line per
    count on stdout. Not part of the benchmark contract line."""
    cfg = inputs.CONFIGS[kind_key]
    kind, T = cfg["kind"], cfg["horizon"]
    pol = inputs.policy_for(kind, cfg["dtype"], cfg["hidden"], seed=0)
    for n in counts:
        dp = wsx.DevicePolicy(pol)
        wsx.autotune(kind, n, dp, T, reps=1, seed=0)
        env = wsx.Env(kind, n, seed=0)
        tr = wsx.Trajectory(kind, T, env.rows)
        ret = torch.empty((T, env.rows), dtype=torch.float32, device="cuda")
        adv = torch.empty_like(ret)
        g = wsx.Grads(dp)
        ws = torch.empty(wsx.ac_grad_workspace_bytes(dp, T * env.rows), dtype=torch.uint8,
                         device="cuda")
        names = ["w1", "b1", "w2", "b2", "w3", "b3"] + ([] if wsx.N_ACTIONS[kind] else ["log_std"])
        master = {k: torch.from_numpy(pol.exact(k).astype("float32")).cuda().reshape(-1)[:dp.tensors[k].numel()]
                  for k in names}
        mom = {k: (torch.zeros_like(v), torch.zeros_like(v)) for k, v in master.items()}

        def roll(i):
            wsx.env_reset(env, epoch=i)
            wsx.rollout(env, dp, T, tr)

        def train(i):
            roll(i)
            wsx.compute_returns(tr, T, 0.99, 0.95, True, torch.float32, ret, adv)
            wsx.ac_grad(dp, wsx.N_ACTIONS[kind], tr.obs.reshape(-1, pol.d_in),
                        tr.action.reshape(-1), ret.reshape(-1), adv.reshape(-1), 0.5, 0.01,
                        grads=g, workspace=ws)
            for k in names:
                wsx.adam_step(master[k], g[k].reshape(-1)[:master[k].numel()], mom[k][0],
                              mom[k][1], i + 1, 3e-4, store=dp.tensors[k].reshape(-1))

        row = {"kind": kind_key.split("_")[0], "envs": n, "horizon": T,
               "shape": wsx.env_shape(env)}
        for name, fn in (("rollout", roll), ("train_iteration", train)):
            fn(0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for i in range(steps):
                fn(i + 1)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            row[name] = {"ms": round(ms, 4), "env_steps_per_s": round(n * T / ms * 1e3, 1)}
        print(json.dumps(row), flush=True)
        del env, tr, ret, adv, ws, g


def strip_comments(text):
    """C/C++ source without its comments and with whitespace runs collapsed,
    so that a change to comments alone keeps the hash below."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_source_hash(csrc=None):
    """Hash of the device-code sources (.hip and .h under csrc/, comments
    left out): counter figures taken on other kernel code are not reported."""
    h = hashlib.sha256()
    csrc = csrc or os.path.join(ROOT, "paper_2408_00930_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if not name.endswith((".hip", ".h")):
            continue
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update(name.encode() + strip_comments(f.read()).encode())
    return h.hexdigest()[:16]


class EnvSet:
    def __init__(self, key, seed, tile_rows, wsx, inputs, torch, shape=None):
        cfg = inputs.CONFIGS[key]
        self.key = key
        self.kind = cfg["kind"]
        self.T = cfg["horizon"]
        self.n_envs = cfg["n_envs"]
        self.policy = inputs.policy_for(self.kind, cfg["dtype"], cfg["hidden"], seed=seed)
        self.dp = wsx.DevicePolicy(self.policy)
        offsets = inputs.agent_offsets(self.n_envs, seed=seed) if self.kind == wsx.MARKET else None
        params = inputs.reaction_params(seed) if self.kind == wsx.REACTION else None
        shape = shape or dict(tile_rows=tile_rows)
        self.env = wsx.Env(self.kind, self.n_envs, seed=seed, agent_offsets=offsets,
                           params=params, **shape)
        self.rows = self.env.rows
        self.traj = wsx.Trajectory(self.kind, self.T, self.rows)
        self.ret = torch.empty((self.T, self.rows), dtype=torch.float32, device="cuda")
        self.adv = torch.empty_like(self.ret)
        self.stream = torch.cuda.Stream()
        self.flop_per_launch = policy_flops(self.policy) * self.rows * (self.T + 1)
        self.k_start, self.k_end = [], []

    def step(self, i, mode, wsx, torch, timed):
        with torch.cuda.stream(self.stream):
            wsx.env_reset(self.env, epoch=i)
            if timed:
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(self.stream)
            wsx.rollout(self.env, self.dp, self.T, self.traj, mode)
            if timed:
                b.record(self.stream)
                self.k_start.append(a)
                self.k_end.append(b)
            wsx.compute_returns(self.traj, self.T, 0.99, 0.95, True, torch.float32,
                                self.ret, self.adv)


def batch_step(sets, i, wsx, torch, timed, k_events, one_launch=True, stream=None):
    """All sets in ONE fused launch on `stream` (default: the first set's
    stream). one_launch: the reset, the roll-out and the returns/GAE of every
    set in that launch (wsx_rollout_batch_ext); else the separate calls (reset
    per set, the batched roll-out, returns per set), the launch alone timed as
    the kernel. k_events None: the caller's events time the launch."""
    st = stream if stream is not None else sets[0].stream
    timed = timed and k_events is not None
    with torch.cuda.stream(st):
        if not one_launch:
            for s in sets:
                wsx.env_reset(s.env, epoch=i)
        if timed:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(st)
        if one_launch:
            wsx.rollout_batch_ext([s.env for s in sets], [s.dp for s in sets], sets[0].T,
                                  [s.traj for s in sets], epoch=i,
                                  returns=[s.ret for s in sets], advantages=[s.adv for s in sets],
                                  gamma=0.99, lam=0.95, bootstrap=True)
        else:
            wsx.rollout_batch([s.env for s in sets], [s.dp for s in sets], sets[0].T,
                              [s.traj for s in sets])
        if timed:
            b.record(st)
            k_events.append((a, b))
        if not one_launch:
            for s in sets:
                wsx.compute_returns(s.traj, s.T, 0.99, 0.95, True, torch.float32, s.ret, s.adv)


def plain_vs_fused(sets, wsx, torch, batched, epoch):
    """One roll-out of every set in the plain per-step form and one in the
    fused form (batched when the benchmark batches), from the same reset: the
    trajectories must be equal bit for bit."""
    fields = ("obs", "action", "reward", "done", "value", "logp", "last_value")

    def run(mode):
        if batched and mode == wsx.MODE_FUSED:   # the timed form: one launch
            wsx.rollout_batch_ext([s.env for s in sets], [s.dp for s in sets], sets[0].T,
                                  [s.traj for s in sets], epoch=epoch,
                                  returns=[s.ret for s in sets], advantages=[s.adv for s in sets],
                                  gamma=0.99, lam=0.95, bootstrap=True)
        else:
            for s in sets:
                wsx.env_reset(s.env, epoch=epoch)
            for s in sets:
                wsx.rollout(s.env, s.dp, s.T, s.traj, mode)
        torch.cuda.synchronize()
        return [[getattr(s.traj, f).clone() for f in fields] for s in sets]

    a, b = run(wsx.MODE_FUSED), run(wsx.MODE_PLAIN)
    equal = all(torch.equal(x, y) for sa, sb in zip(a, b) for x, y in zip(sa, sb))
    # the sets' returns again match their (last written) trajectories
    for s in sets:
        wsx.compute_returns(s.traj, s.T, 0.99, 0.95, True, torch.float32, s.ret, s.adv)
    torch.cuda.synchronize()
    return {"plain_equals_fused": bool(equal), "epoch": epoch, "fields": list(fields)}


def peak_probe(torch):
    """Achievable rates on this GPU, for reading the roofline fractions: a
    device-to-device copy of 4 GiB (HBM read + write) and 8192^3 matrix products
    in BF16 and FP32 through torch (hipBLASLt / rocBLAS)."""
    out = {}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps * 1e-3

    n = 4 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    t = timed(lambda: dst.copy_(src), 5)
    out["hbm_copy_gb_s"] = round(2 * n / t / 1e9, 1)
    del src, dst
    m = 8192
    for name, dt in (("bf16_gemm_tflops", torch.bfloat16), ("fp32_gemm_tflops", torch.float32)):
        x = torch.randn(m, m, device="cuda").to(dt)
        y = torch.randn(m, m, device="cuda").to(dt)
        t = timed(lambda: torch.matmul(x, y), 10)
        out[name] = round(2 * m ** 3 / t / 1e12, 1)
        del x, y
    torch.cuda.empty_cache()
    return out


def run_form(sets, mode, steps, warmup, wsx, torch, first_epoch, batched=False, one_launch=True):
    main = torch.cuda.current_stream()
    k_events = []

    # A batched step is one launch (or, without one_launch, the launch with
    # its reset and returns kernels) on the main stream, as a training loop
    # would enqueue it: a second stream adds two cross-stream waits per step
    # (~25 us). With one_launch the step's own events time the launch.
    def one(i, timed):
        if batched:
            batch_step(sets, i, wsx, torch, timed, None if one_launch else k_events,
                       one_launch, stream=main)
            return
        for s in sets:
            s.stream.wait_stream(main)
            s.step(i, mode, wsx, torch, timed=timed)
        for s in sets:
            main.wait_stream(s.stream)

    for i in range(warmup):
        one(first_epoch + i, False)
    for s in sets:
        s.k_start, s.k_end = [], []
    torch.cuda.synchronize()
    step_ev = []
    t0 = time.perf_counter()
    for i in range(steps):
        a = torch.cuda.Event(enable_timing=True)
        a.record(main)
        one(first_epoch + warmup + i, True)
        b = torch.cuda.Event(enable_timing=True)
        b.record(main)
        step_ev.append((a, b))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lat = sorted(a.elapsed_time(b) for a, b in step_ev)
    if batched:
        kern = {"batch": [a.elapsed_time(b) for a, b in (step_ev if one_launch else k_events)]}
    else:
        kern = {s.key: [a.elapsed_time(b) for a, b in zip(s.k_start, s.k_end)] for s in sets}
    return elapsed, lat, kern


def percentile(sorted_vals, q):
    if not sorted_vals:
        return None
    k = min(len(sorted_vals) - 1, max(0, int(round(q / 100.0 * (len(sorted_vals) - 1)))))
    return sorted_vals[k]


def iqr(sorted_vals, digits):
    """Interquartile range of sorted values (None when there are none)."""
    if not sorted_vals:
        return None
    return round(percentile(sorted_vals, 75) - percentile(sorted_vals, 25), digits)


def cpu_baseline(sets, sample_envs, single_thread=True):
    """The FP64 oracle on a bounded sample of the same workload (the first
    `sample_envs` envs of each set over the full horizon); with single_thread
    also on one thread over a quarter of that sample."""
    import numpy as np

    import oracle as O
    from paper_2408_00930_amd import inputs

    def run(envs):
        total = 0
        t0 = time.perf_counter()
        for s in sets:
            n = min(envs, s.n_envs)
            offsets = inputs.agent_offsets(s.n_envs, seed=0)[:n + 1] if s.kind == O.MARKET else None
            params = inputs.reaction_params(0).astype(np.float64) if s.kind == O.REACTION else None
            oenv = O.env_hold(s.kind, n, offsets, params)
            st = O.env_reset(oenv, 0, 0)
            out = O.rollout(oenv, O.mlp_hold(s.policy), 0, 0, 0, s.T, st,
                            s.policy.exact("log_std"), margins=False)
            O.returns_gae(out["reward"], out["value"], out["done"], out["last_value"], 0.99, 0.95)
            total += n * s.T
        return total, time.perf_counter() - t0

    def median_of_3(envs):
        runs = sorted((run(envs) for _ in range(3)), key=lambda r: r[1])
        return runs[1]

    cores = O.num_threads()
    total_env_steps, el = median_of_3(sample_envs)
    out = {"value": total_env_steps / el, "unit": "env-steps/s", "cores": cores,
           "kind": "oracle",
           "sample": f"first {sample_envs} envs of each set over the full horizon "
                     f"({total_env_steps} env-steps, median of 3 runs: {el:.1f} s), FP64 C "
                     f"oracle with OpenMP over envs, returns/GAE included",
           "cpu": cpu_model()}
    if single_thread:
        # the same oracle on one thread, over a quarter of the sample
        O.set_threads(1)
        one_steps, one_el = median_of_3(max(1, sample_envs // 4))
        O.set_threads(cores)
        out["single_thread"] = {"value": round(one_steps / one_el, 1), "cores": 1,
                                "sample": f"first {max(1, sample_envs // 4)} envs of each set "
                                          f"({one_steps} env-steps, median of 3 runs: "
                                          f"{one_el:.1f} s)"}
    return out


def cpu_model():
    """The host CPU's model name, from /proc/cpuinfo (None if unreadable)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def serving(args, wsx, inputs, torch):
    """Poisson arrivals of roll-out requests into the continuous-batching
    server: kind uniform over Pendulum, Acrobot, market, reaction; replicas
    log-uniform in [64, 8192]; horizon uniform in [10, 500]."""
    import math
    import threading

    import numpy as np
    kinds = [wsx.PENDULUM, wsx.ACROBOT, wsx.MARKET, wsx.REACTION]
    cfg = {wsx.PENDULUM: ("bf16", 256), wsx.ACROBOT: ("bf16", 256), wsx.MARKET: ("bf16", 256),
           wsx.REACTION: ("fp8", 512)}
    pols = {k: wsx.DevicePolicy(inputs.policy_for(k, cfg[k][0], cfg[k][1], seed=k)) for k in kinds}
    params = torch.from_numpy(inputs.reaction_params(0)).cuda()
    rng = np.random.default_rng(args.serve_seed)
    n_total = args.serve_warmup + args.serve_requests
    specs = []
    for i in range(n_total):
        k = kinds[int(rng.integers(0, 4))]
        n = int(round(math.exp(rng.uniform(math.log(64), math.log(8192)))))
        T = int(rng.integers(10, 501))
        gap = rng.exponential(1.0 / args.serve_rate)
        specs.append((k, n, T, gap))
    srv = wsx.Server(int(args.serve_arena_gb * (1 << 30)), chunk_steps=args.serve_chunk,
                     max_batch=64)
    ids = [None] * n_total
    t_sub = [0.0] * n_total

    def submitter():
        t_next = time.perf_counter()
        for i, (k, n, T, gap) in enumerate(specs):
            t_next += gap
            delay = t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            kw = {}
            if k == wsx.MARKET:
                kw["agent_offsets"] = inputs.agent_offsets(n, seed=i)
            if k == wsx.REACTION:
                kw["params"] = params
            t_sub[i] = time.perf_counter()
            ids[i] = srv.submit(k, pols[k], T, n_envs=n, seed=i, **kw)

    th = threading.Thread(target=submitter)
    th.start()
    lat, steps, t_done = [], 0, []
    for i in range(n_total):
        while ids[i] is None:
            time.sleep(1e-4)
        r = srv.wait(ids[i], -1)
        t_done.append(time.perf_counter())
        if i >= args.serve_warmup:
            lat.append(r.latency_ms)
            steps += specs[i][1] * specs[i][2]
        srv.release(ids[i])
        if (i + 1) % 200 == 0:
            print(f"[bench] serving: {i + 1}/{n_total} requests done", file=sys.stderr, flush=True)
    th.join()
    st = srv.stats()
    srv.close()
    span = t_done[-1] - t_sub[args.serve_warmup]
    lat.sort()
    return {"requests": args.serve_requests, "warmup_requests": args.serve_warmup,
            "rate_per_s": args.serve_rate, "arena_gb": args.serve_arena_gb,
            "chunk_steps": args.serve_chunk,
            "latency_ms": {"p50": round(percentile(lat, 50), 3), "p99": round(percentile(lat, 99), 3),
                           "max": round(lat[-1], 3)},
            "env_steps_per_s": round(steps / span, 1), "makespan_s": round(span, 3),
            "launches": st["launches"], "arena_peak_gb": round(st["arena_peak"] / 2**30, 2)}


def counters_for(kernel_name):
    """The committed rocprofv3 counter figures of a kernel, if they were taken
    on the current kernel sources (else an empty dict)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    ent = data.get(kernel_name)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return {}
    return ent


def traffic_for(kernel_name, launches_bytes_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary."""
    return counters_for(kernel_name).get(launches_bytes_key)


def unit_busy_for(kernel_name):
    """Share of the dispatch's cycles the MFMA and vector ALUs were busy
    (rocprofv3 SQ_VALU_MFMA_BUSY_CYCLES and SQ_ACTIVE_INST_VALU over
    GRBM_GUI_ACTIVE), or None."""
    ent = counters_for(kernel_name)
    if "mfma_busy" not in ent:
        return None
    return {"mfma": ent["mfma_busy"], "valu": ent["valu_busy"],
            "from": "rocprofv3 PMC: SQ_VALU_MFMA_BUSY_CYCLES, SQ_ACTIVE_INST_VALU / GRBM_GUI_ACTIVE"}


def measure(workload, args, wsx, inputs, torch, plain_steps, cpu_envs, single_thread):
    """One workload: the autotuner's shape (untimed), then the fused form
    timed over args.steps steps after args.warmup, the plain / graph / fused
    graph forms, plain = fused bit for bit on the same inputs, the roofline
    of the fused launch and the oracle on a bounded sample. Returns the
    record and the sets."""
    keys = WORKLOADS[workload]
    # one fused launch per step for all sets (a single set is a batch of one)
    batched = len(keys) == 1 or not args.no_batch
    tuned = {}
    shape = dict(zip(("tile_rows", "waves", "occupancy"),
                     (int(x) for x in args.shape.split(",")))) if args.shape else None
    if args.autotune and not args.tile_rows and not shape:
        # the library's autotuner picks the kernel shape (untimed here): for a
        # batched workload one shape for the whole single launch
        spec = []
        for key in keys:
            cfg = inputs.CONFIGS[key]
            kind = cfg["kind"]
            spec.append(dict(
                kind=kind, n_envs=cfg["n_envs"], seed=0, horizon=cfg["horizon"],
                policy=wsx.DevicePolicy(inputs.policy_for(kind, cfg["dtype"], cfg["hidden"], seed=0)),
                agent_offsets=inputs.agent_offsets(cfg["n_envs"], seed=0)
                if kind == wsx.MARKET else None,
                params=inputs.reaction_params(0) if kind == wsx.REACTION else None))
        t0 = time.perf_counter()
        if batched:
            # median of five timed roll-outs per candidate: with two, a hot
            # clock after the previous workload has flipped kernels 6 % apart
            tuned["batch"] = wsx.autotune_batch(spec, spec[0]["horizon"], reps=5)
        else:
            for key, d in zip(keys, spec):
                tuned[key] = wsx.autotune(d["kind"], d["n_envs"], d["policy"], d["horizon"], reps=5,
                                          seed=0, agent_offsets=d["agent_offsets"],
                                          params=d["params"])
        print(f"[bench] {workload} autotune: {tuned} in {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    sets = [EnvSet(k, 0, args.tile_rows, wsx, inputs, torch, shape) for k in keys]
    env_steps = sum(s.n_envs * s.T for s in sets)
    forms = args.forms.split(",")

    result = {}
    el, lat, kern = run_form(sets, wsx.MODE_FUSED, args.steps, args.warmup, wsx, torch, 0,
                             batched=batched)
    result["fused"] = (el, lat, kern)
    print(f"[bench] {workload} fused: {args.steps} steps in {el:.3f} s", file=sys.stderr,
          flush=True)
    if batched and "fused_calls" in forms:
        # the same launch without the reset and returns in it: reset and
        # returns as separate kernels around it
        r = run_form(sets, wsx.MODE_FUSED, args.steps, 5, wsx, torch, 2000, batched=True,
                     one_launch=False)
        result["fused_calls"] = r + (args.steps,)
        print(f"[bench] {workload} fused_calls: {args.steps} steps in {r[0]:.3f} s",
              file=sys.stderr, flush=True)
    for name, mode in (("plain", wsx.MODE_PLAIN), ("graph", wsx.MODE_GRAPH),
                       ("fused_graph", wsx.MODE_FUSED_GRAPH)):
        n = args.steps if name == "fused_graph" else plain_steps
        if name in forms and n > 0:
            r = run_form(sets, mode, n, 1, wsx, torch, 1000)
            result[name] = r + (n,)
            print(f"[bench] {workload} {name}: {n} steps in {r[0]:.3f} s", file=sys.stderr,
                  flush=True)

    # plain and fused forms on identical inputs, compared in the same run
    parity = None
    if "plain" in forms and plain_steps > 0:
        parity = plain_vs_fused(sets, wsx, torch, batched, epoch=4321)
        print(f"[bench] {workload} parity: {parity}", file=sys.stderr, flush=True)

    el, lat, kern = result["fused"]
    value = env_steps * args.steps / el
    # dominant kernel: the fused roll-out launch (the batched one, or the set's
    # launch with the most total time)
    if batched:
        avg_ms = sum(kern["batch"]) / len(kern["batch"])
        flop = sum(s.flop_per_launch for s in sets)
        dtype = sets[0].policy.dtype
        kname = f"k_fused/{workload}"
    else:
        dom = max(sets, key=lambda s: sum(kern[s.key]))
        avg_ms = sum(kern[dom.key]) / len(kern[dom.key])
        flop = dom.flop_per_launch
        dtype = dom.policy.dtype
        kname = f"k_fused/{dom.key}"
    achieved = flop / (avg_ms * 1e-3) / 1e12
    # one wave per replica (tile of one row, one wave): the policy runs as FP32
    # FMAs on the vector ALU, whose FP32 peak is the same 157.3 TFLOP/s
    row_wave = all(wsx.env_shape(s.env)[:2] == (1, 1) for s in sets)
    roofline = {"bound": "alu" if row_wave else "mfma", "achieved": round(achieved, 2), "peak": PEAK_TFLOPS[dtype],
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[dtype], 4),
                "traffic": traffic_for(kname, "hbm_bytes_per_launch"),
                "unit_busy": unit_busy_for(kname),
                "kernel": kname, "avg_launch_ms": round(avg_ms, 4),
                "flop_per_launch": flop}
    out = {
        "value": round(value, 1), "unit": "env-steps/s",
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(el / args.steps * 1e3, 4),
        "dtype": "bf16" if any(s.policy.dtype == "bf16" for s in sets) else dtype,
        "config": {"workload": workload, "envs": sum(s.n_envs for s in sets),
                   "rows": sum(s.rows for s in sets),
                   "horizon": max(s.T for s in sets), "sets": [s.key for s in sets],
                   "policy": {s.key: f"{s.policy.dtype} {s.policy.d_in}-{s.policy.h1}-"
                                     f"{s.policy.h2}-{s.policy.n_head}" for s in sets},
                   "returns": "FP64, FP32 outputs" + (", in the roll-out launch" if batched
                                                         else ", separate kernel"),
                   "reset": "in the roll-out launch" if batched else "separate kernel",
                   "streams": 1 if batched else len(sets),
                   "kernel_shape": {s.key: dict(zip(("tile_rows", "waves", "occupancy",
                                                     "chunk_steps"), wsx.env_shape(s.env)))
                                    for s in sets},
                   "autotuned": bool(tuned), "one_launch": batched,
                   "tiles": {s.key: dict(zip(("tiles", "rows_per_tile"), s.env.tiles()),
                                         fill=round(s.rows / (s.env.tiles()[0] *
                                                              s.env.tiles()[1]), 4))
                             for s in sets}},
        "latency_ms": {"p50": round(percentile(lat, 50), 4), "p99": round(percentile(lat, 99), 4),
                       "iqr": iqr(lat, 4)},
        "roofline": roofline,
    }
    if any(s.kind == wsx.MARKET for s in sets):
        agent_steps = sum(s.rows * s.T for s in sets)
        out["agent_steps_per_s"] = round(agent_steps * args.steps / el, 1)
    for name in ("fused_calls", "plain", "graph", "fused_graph"):
        if name in result:
            pel, plat, pk, n = result[name]
            pv = env_steps * n / pel
            out[name] = {"value": round(pv, 1), "steps": n, "ms_per_step": round(pel / n * 1e3, 3),
                         "latency_ms": {"p50": round(percentile(plat, 50), 3),
                                        "p99": round(percentile(plat, 99), 3),
                                        "iqr": iqr(plat, 3)}}
            if name == "fused_calls":
                out[name]["avg_launch_ms"] = round(sum(pk["batch"]) / len(pk["batch"]), 4)
            out[f"fused_speedup_vs_{name}"] = round(value / pv, 3 if name == "fused_calls" else 2)
    if parity is not None:
        out["parity"] = parity
    if cpu_envs > 0 and not args.no_cpu_baseline:
        print(f"[bench] {workload} cpu baseline: the oracle on {cpu_envs} envs of each set",
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(sets, cpu_envs, single_thread)
        print(f"[bench] {workload} cpu baseline: {out['cpu_baseline']['value']:.4g} env-steps/s",
              file=sys.stderr, flush=True)
    return out, sets


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 20 untimed steps bring the GPU to its sustained clock (after 3, launches
    # still ran ~6 % slower); 50 timed steps are ~55 ms of GPU work
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--workload", default="pendulum_acrobot_10k", choices=sorted(WORKLOADS))
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--shape", default="",
                    help="ROWS,WAVES,OCCUPANCY kernel shape for every set (skips the autotuner)")
    ap.add_argument("--cpu-sample-envs", type=int, default=0,
                    help="envs of each set the oracle runs for the CPU baseline (0: the "
                         "workload's default, about 1-5 s of oracle work)")
    ap.add_argument("--also", default="cartpole_1k,market_2k,reaction_4k",
                    help="other workloads measured the same way, reported as sub-records "
                         "under 'workloads' ('' for none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--forms", default="fused,fused_calls,plain,graph,fused_graph")
    ap.add_argument("--no-batch", action="store_true",
                    help="run a multi-set workload as one launch per set on its own stream")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="run the built-in default kernel shapes instead of the autotuner's")
    ap.add_argument("--update-steps", type=int, default=5,
                    help="timed passes of the actor-critic update after the roll-out legs "
                         "(0: skip)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="measured requests of the serving load (0: skip serving)")
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-arena-gb", type=float, default=200.0)
    ap.add_argument("--serve-chunk", type=int, default=25)
    ap.add_argument("--serve-seed", type=int, default=0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic for scaling HBM byte counters)")
    ap.add_argument("--sweep", default="",
                    help="instead of the benchmark: env-count sweep of this workload key "
                         "(e.g. pendulum_10k), one JSON line per count")
    ap.add_argument("--sweep-counts", default="10,100,1000,10000,100000,1000000")
    ap.add_argument("--peak-probe", action="store_true",
                    help="instead of the benchmark: achievable HBM copy bandwidth and BF16 / "
                         "FP32 GEMM rates on this GPU, one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (replicas "
              "would shard by contiguous env ranges with no exchange). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2408_00930_amd import inputs, wsx
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    wsx.lib()
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.sweep:
        sweep(args.sweep, [int(x) for x in args.sweep_counts.split(",")], args.steps, wsx, inputs,
              torch)
        return
    if args.peak_probe:
        print(json.dumps({"peak_probe": peak_probe(torch),
                          "published": {"hbm_gb_s": 8000, "bf16_tflops": 2500,
                                        "fp32_tflops": 157.3}}), flush=True)
        return
    headline, sets = measure(args.workload, args, wsx, inputs, torch, args.plain_steps,
                             args.cpu_sample_envs or CPU_SAMPLE_ENVS[args.workload], True)
    out = {"metric": METRIC, "value": headline["value"], "unit": "env-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": headline["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": headline["dtype"], "data": "synthetic (seeded inputs; random-init policies)"}
    for k, v in headline.items():
        if k not in out:
            out[k] = v
    # the other workloads, each timed the same way, as sub-records
    others = [w for w in args.also.split(",") if w and w != args.workload]
    if others:
        out["workloads"] = {}
    for w in others:
        rec, _ = measure(w, args, wsx, inputs, torch, args.plain_steps,
                         CPU_SAMPLE_ENVS.get(w, 64), False)
        out["workloads"][w] = rec
    if args.serve_requests > 0:
        out["serving"] = serving(args, wsx, inputs, torch)
    if args.update_steps > 0:   # last: it writes new weights into the policies
        upd = update_leg(sets, args.update_steps, wsx, torch)
        if upd:
            out["update"] = upd
            print(f"[bench] update: {upd['ms_per_update']} ms per update", file=sys.stderr,
                  flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

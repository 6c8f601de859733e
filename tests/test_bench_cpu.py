"""Host logic of bench.py that runs without a GPU: the latency statistics,
the oracle's CPU baseline leg, and the single-GPU guard."""
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_percentile_and_iqr():
    v = sorted([5.0, 1.0, 4.0, 2.0, 3.0])
    assert bench.percentile(v, 50) == 3.0
    assert bench.percentile(v, 0) == 1.0 and bench.percentile(v, 100) == 5.0
    assert bench.iqr(v, 3) == 2.0
    assert bench.percentile([], 50) is None and bench.iqr([], 3) is None


def test_cpu_baseline_reports_all_threads_and_one():
    """A tiny sample of a CartPole set: the leg returns the oracle's rate at
    its thread count and at one thread, and restores the thread count."""
    import oracle as O
    from paper_2408_00930_amd import inputs
    cfg = inputs.CONFIGS["cartpole_1k"]
    s = types.SimpleNamespace(kind=cfg["kind"], n_envs=cfg["n_envs"], T=20,
                              policy=inputs.policy_for(cfg["kind"], cfg["dtype"], cfg["hidden"], seed=0))
    before = O.num_threads()
    out = bench.cpu_baseline([s], 8)
    assert O.num_threads() == before
    assert out["kind"] == "oracle" and out["unit"] == "env-steps/s"
    assert out["value"] > 0 and out["cores"] == before
    assert out["single_thread"]["cores"] == 1 and out["single_thread"]["value"] > 0
    assert "160 env-steps" in out["sample"] and "40 env-steps" in out["single_thread"]["sample"]
    assert out["cpu"] is None or isinstance(out["cpu"], str)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr


def test_source_hash_ignores_comments_only(tmp_path):
    """Profile figures stay valid across comment edits, not code edits."""
    assert bench.strip_comments("a = 1; // x\n/* y\n z */ b  =\n2;") == "a = 1; b = 2;"
    (tmp_path / "k.hip").write_text("int f() { return 1; } // one\n")
    (tmp_path / "notes.txt").write_text("not device code")
    h0 = bench.kernel_source_hash(str(tmp_path))
    (tmp_path / "k.hip").write_text("/* the first */\nint f() {\n  return 1;  // still one\n}\n")
    assert bench.kernel_source_hash(str(tmp_path)) == h0
    (tmp_path / "k.hip").write_text("int f() { return 2; }\n")
    assert bench.kernel_source_hash(str(tmp_path)) != h0

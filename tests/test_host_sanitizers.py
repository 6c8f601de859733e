"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):

- the roll-out server's arena and admission order (admission.h) with a fake
  clock and a fake arena, checked against a byte map of owners;
- the FP64 oracle driven through every entry point on every kind;
- the C ABI's host paths (validation, sizes, the tuning table's text format,
  the server's checks) with the library's host code built with the
  sanitizers (-Xarch_host: the device code is built as usual).

Each driver is a separate program built here; a sanitizer report or a failed
check ends it with a nonzero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
CSRC = os.path.join(ROOT, "paper_2408_00930_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, cwd, timeout):
    res = subprocess.run(cmd, cwd=cwd, capture_output=True, text=True, timeout=timeout, env=ENV)
    assert res.returncode == 0, f"{' '.join(cmd[:3])} ...\n{res.stdout[-3000:]}\n{res.stderr[-3000:]}"
    return res.stdout


def test_admission_and_arena_under_sanitizers(tmp_path):
    exe = str(tmp_path / "admission_test")
    _run(["g++", "-std=c++17", *SAN, "-I", CSRC, os.path.join(HOST, "admission_test.cpp"), "-o",
          exe], ROOT, 120)
    assert "admission: ok" in _run([exe], ROOT, 120)


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    _run(["gcc", "-std=c11", *SAN, "-fopenmp", "-ffp-contract=off",
          os.path.join(HOST, "oracle_sanitize.c"), "-o", exe, "-lm"], ROOT, 120)
    assert "oracle under sanitizers: ok" in _run([exe], ROOT, 300)


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="the HIP toolchain builds the library's host code")
def test_abi_host_paths_under_sanitizers(tmp_path):
    from paper_2408_00930_amd import build as B
    objs = [os.path.join(B.BUILD, f + ".o") for f in ("rollout.hip", "returns.hip", "update.hip")]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    hipcc = B.hipcc()
    host = []
    for src in ("abi.cpp", "serve.cpp", "tune.cpp", "compose.cpp"):
        o = str(tmp_path / (src + ".o"))
        # the sanitizers instrument the host half only (-Xarch_host before each)
        _run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-Xarch_host", "-fno-sanitize-recover=all", "-Xclang", "-target-feature", "-Xclang",
              "-packed-fp32-ops", "-I", B.INCLUDE, "-x", "hip", "-c", os.path.join(CSRC, src),
              "-o", o], ROOT, 300)
        host.append(o)
    clang = "/opt/rocm/llvm/bin/clang++"
    exe = str(tmp_path / "abi_sanitize")
    _run([clang, "-std=c++17", "-g", "-fsanitize=address,undefined", "-I", B.INCLUDE,
          os.path.join(HOST, "abi_sanitize.cpp"), *host, *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib", "-o", exe], ROOT, 300)
    assert "abi host paths under sanitizers: ok" in _run([exe, str(tmp_path)], ROOT, 300)

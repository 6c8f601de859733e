"""Build libwsx.so (gfx950) in-tree with hipcc.

    python -m paper_2408_00930_amd.build

Every HIP source is compiled for gfx950 only; packed FP32 instructions are
disabled in the device code; floating-point contraction is limited to single
expressions so that every kernel that inlines a device function rounds it the
same way.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libwsx.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

SOURCES = ["rollout.hip", "returns.hip", "update.hip", "abi.cpp", "serve.cpp", "tune.cpp",
           "compose.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
         "-Wall", "-Wno-unused-variable", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", INCLUDE]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the HIP toolchain is required to build libwsx")
    return path


# The roll-out kernels keep their weights in registers; with the matrix-core
# accumulators in VGPRs (not AGPRs) the tanh epilogue reads them without a
# v_accvgpr_read per value (one vector instruction in six of the epilogue).
SOURCE_FLAGS = {"rollout.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ([hipcc()] + FLAGS + SOURCE_FLAGS.get(src, []) +
           ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{err}")
    return obj


def build() -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lhiprtc"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"linking libwsx.so failed:\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

"""Build libmcx.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1711_03244_amd.build          # always rebuilds
    python -m paper_1711_03244_amd.build --if-stale
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmcx.so")
MICROBENCH = os.path.join(HERE, "mcx_microbench")
SOURCES = ["mcx_transport.hip", "mcx_tally.hip", "mcx_detpost.hip", "mcx_runtime.hip",
           "nn_kernels.hip", "nn_runtime.hip"]
HEADERS = ["mcx_internal.hpp", "mcx_detpost.hpp", "nn_internal.hpp", os.path.join("..", "..", "include", "mcx.h"),
           os.path.join("..", "..", "include", "mcx_nn.h")]
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    h = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(h):
        raise RuntimeError("hipcc not found; ROCm is required to build libmcx")
    return h


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, s) for s in SOURCES + HEADERS]
    return any(os.path.getmtime(d) > t for d in deps)


def build(force: bool = True, extra=()) -> str:
    if not force and not stale():
        return LIB
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + FLAGS + list(extra) + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    subprocess.run(cmd, check=True, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


def build_microbench() -> str:
    """Standalone atomic / VALU / Philox microbenchmark (prints JSON lines)."""
    src = os.path.join(CSRC, "microbench.hip")
    tmp = MICROBENCH + ".tmp"
    flags = [f for f in FLAGS if f not in ("-fPIC", "-shared")]
    subprocess.run([hipcc()] + flags + ["-o", tmp, src], check=True, cwd=CSRC)
    os.replace(tmp, MICROBENCH)
    return MICROBENCH


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
    print(build_microbench())

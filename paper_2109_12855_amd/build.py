"""Build the gfx950 shared library ``libsdeliver.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsdeliver.so")
CPU_LIB = os.path.join(HERE, "libsdcpu.so")
CPU_SOURCES = [os.path.join(HERE, "cpu", "sd_cpu.c")]
SOURCES = [os.path.join(CSRC, "sd_api.cpp"), os.path.join(CSRC, "sd_autotune.cpp"),
           os.path.join(CSRC, "sd_kernels.hip"), os.path.join(CSRC, "sd_noalloc.hip")]
ARCH = os.environ.get("SD_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libsdeliver.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "'-packed-fp32-ops' is not a recognized feature"
    msgs = [l for l in (res.stdout + res.stderr).splitlines() if noise not in l]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    build_cpu()
    return LIB


def build_cpu() -> str:
    """Compile the multithreaded CPU delivery comparator into libsdcpu.so."""
    tmp = CPU_LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-o", tmp,
           *CPU_SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("gcc failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, CPU_LIB)
    return CPU_LIB


if __name__ == "__main__":
    print(build(verbose=True))

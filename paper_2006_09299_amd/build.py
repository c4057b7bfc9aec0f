"""Compile libccl.so (HIP, gfx950) in-tree with hipcc, and the host LSL-BW
(liblslbw.so) with g++."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libccl.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["ccl.hip", "ccl_server.cpp"]  # kernels + C-ABI; serving front end (host code)
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


HOST_SRC = os.path.join(HERE, "host", "lsl_bw.cpp")
HOST_LIB = os.path.join(HERE, "host", "liblslbw.so")


def build_host() -> str:
    """liblslbw.so: the single-thread host LSL-BW (plain g++, no GPU code)."""
    tmp = HOST_LIB + ".tmp"
    subprocess.check_call(["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall", "-Wextra", HOST_SRC, "-o", tmp])
    os.replace(tmp, HOST_LIB)
    return HOST_LIB


def build() -> str:
    build_host()
    srcs = [os.path.join(CSRC, f) for f in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *srcs, "-o", tmp]
    p = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the gfx feature flag; that warning is harmless
    noise = [ln for ln in p.stderr.splitlines() if ln.strip() and "packed-fp32-ops" not in ln]
    if p.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(noise))
    if noise:
        sys.stderr.write("\n".join(noise) + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

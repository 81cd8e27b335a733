"""Build libnbs.so for gfx950 in-tree with hipcc (no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libnbs.so")
SOURCES = ["kernels.hip", "plan.cpp", "compiler.cpp", "static_path.hip"]
ARCH = os.environ.get("NBS_OFFLOAD_ARCH", "gfx950")


def hipcc_cmd(out: str):
    return [
        "hipcc", "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed FP32 instructions are kept out of every kernel
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wno-unused-command-line-argument",
        "-I", os.path.join(ROOT, "include"), "-I", CSRC,
        "-o", out,
    ] + [os.path.join(CSRC, s) for s in SOURCES]


SYNTH_SOURCE = "synth.hip"
SYNTH_LIB = os.path.join(LIBDIR, "libnbs_synth.so")


def build_synth(verbose: bool = False) -> str:
    """The device generator of the synthetic inputs (a library of its own:
    input generation, not part of the method's path)."""
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = SYNTH_LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument",
           "-o", tmp, os.path.join(CSRC, SYNTH_SOURCE)]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libnbs_synth.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, SYNTH_LIB)
    return SYNTH_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = hipcc_cmd(tmp)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libnbs.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    build_synth(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

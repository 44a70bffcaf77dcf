"""Build the gfx950 HIP library libafqmc.so in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libafqmc.so")
SOURCES = ["kernels.hip", "qroute.hip", "multidet.hip", "bf16.hip", "abi.cpp", "stats.cpp"]
ARCH = os.environ.get("AFQMC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_commands(out: str):
    # Packed FP32 instructions are disabled for all device code.
    flags = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src + ".o")
        cmds.append([hipcc(), *flags, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # no undefined symbols: a declaration without a definition fails here, not at load
    cmds.append([hipcc(), f"--offload-arch={ARCH}", "-shared", "-Wl,--no-undefined", *objs, "-o", out])
    return cmds


def build(verbose: bool = False) -> str:
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    tmp = LIB + ".tmp"
    for cmd in compile_commands(tmp):
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("HIP build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

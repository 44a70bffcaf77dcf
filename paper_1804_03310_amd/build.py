"""Build the gfx950 HIP library libafqmc.so in-tree with hipcc.

`build()` always recompiles.  `ensure_built()` compiles only when the library
is missing or was built from other sources: beside the library a stamp file
holds the SHA-256 of every source, header and compile flag it was built from,
so a fresh checkout (no library) and an edited source both lead to one build
before the first load, and an up-to-date library is loaded as it is.
"""
from __future__ import annotations

import concurrent.futures as cf
import fcntl
import hashlib
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libafqmc.so")
STAMP = LIB + ".sha256"
SOURCES = ["kernels.hip", "qroute.hip", "multidet.hip", "bf16.hip", "resident.hip", "noalloc.hip",
           "abi.cpp", "stats.cpp"]
ARCH = os.environ.get("AFQMC_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags():
    # Packed FP32 instructions are disabled for all device code.
    return ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]


def _inputs():
    """Every file the library is built from, in a fixed order."""
    names = sorted(set(SOURCES) | {f for f in os.listdir(CSRC)
                                   if f.endswith((".hpp", ".h", ".hip", ".cpp"))})
    return [os.path.join(CSRC, f) for f in names] + [os.path.join(INCLUDE, f)
                                                     for f in sorted(os.listdir(INCLUDE))]


def source_digest() -> str:
    """SHA-256 over the flags and every input file.  Paths enter relative to
    the repository root, so a copy of the tree elsewhere (same sources) finds
    its shipped library current."""
    h = hashlib.sha256()
    flags = [os.path.relpath(f, ROOT) if f in (INCLUDE, CSRC) else f for f in _flags()]
    h.update(" ".join(flags + SOURCES).encode())
    for p in _inputs():
        h.update(os.path.relpath(p, ROOT).encode())
        with open(p, "rb") as f:
            h.update(hashlib.sha256(f.read()).digest())
    return h.hexdigest()


def compile_commands(out: str):
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src + ".o")
        cmds.append([hipcc(), *_flags(), "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    # no undefined symbols: a declaration without a definition fails here, not at load
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-Wl,--no-undefined", *objs, "-o", out]
    return cmds, link


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("HIP build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link libafqmc.so; write the stamp."""
    os.makedirs(os.path.join(CSRC, "_build"), exist_ok=True)
    digest = source_digest()
    tmp = LIB + ".tmp%d" % os.getpid()
    cmds, link = compile_commands(tmp)
    workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with cf.ThreadPoolExecutor(workers) as pool:
        for fut in [pool.submit(_run, c, verbose) for c in cmds]:
            fut.result()
    _run(link, verbose)
    os.replace(tmp, LIB)
    with open(STAMP + ".tmp", "w") as f:
        f.write(digest + "\n")
    os.replace(STAMP + ".tmp", STAMP)
    return LIB


def is_current() -> bool:
    if not (os.path.exists(LIB) and os.path.exists(STAMP)):
        return False
    with open(STAMP) as f:
        return f.read().strip() == source_digest()


def ensure_built() -> str:
    """Build libafqmc.so if it is missing or stale; one process builds at a
    time (an advisory lock beside the library), the others wait and reuse it."""
    if is_current():
        return LIB
    with open(LIB + ".lock", "w") as lk:
        fcntl.flock(lk, fcntl.LOCK_EX)
        try:
            if not is_current():
                print(f"[afqmc] building {LIB} for {ARCH} (missing or stale) ...", file=sys.stderr,
                      flush=True)
                t0 = time.perf_counter()
                build()
                print(f"[afqmc] built in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                      flush=True)
        finally:
            fcntl.flock(lk, fcntl.LOCK_UN)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Build librl0.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1704_09012_amd.build        # or build() from Python

Every call recompiles.  The library lands next to this file, where the binding loads it.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "librl0.so")
# the same library with the loop kernels' index checks compiled in (rl0_device_check)
CHECKED_OUT = os.path.join(HERE, "librl0_checked.so")
CHECKED_SOURCES = ("kernels.hip", "batched.hip", "mlp.hip")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["constants.cpp", "general.cpp", "rl0.cpp", "kernels.hip", "batched.hip", "mlp.hip", "noalloc.hip"]

COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-ffp-contract=off",
    # keep the compiler from forming packed fp32 instructions (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, checked: bool = False) -> str:
    obj = os.path.join(BUILD_DIR, src + (".checked.o" if checked else ".o"))
    path = os.path.join(CSRC, src)
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    defs = ["-DRL0_DEVICE_CHECKS=1"] if checked else []
    cmd = [_hipcc(), *COMMON, *defs, *lang, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, out: str) -> None:
    tmp = out + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Builds librl0.so and librl0_checked.so (the latter differs only in the loop
    kernels, the batched kernel and the network kernel, compiled with their index checks)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = [(src, False) for src in SOURCES] + [(src, True) for src in CHECKED_SOURCES]
    # the compiles of the largest sources first, so that they overlap the others
    jobs.sort(key=lambda j: j[0] not in CHECKED_SOURCES)
    with ThreadPoolExecutor(max_workers=max(1, min(8, len(os.sched_getaffinity(0))))) as ex:
        done = dict(zip(jobs, ex.map(lambda j: _compile(*j), jobs)))
    objs = [done[(src, False)] for src in SOURCES]
    _link(objs, OUT)
    _link([done[(src, src in CHECKED_SOURCES)] for src in SOURCES], CHECKED_OUT)
    if verbose:
        print("built", OUT, "and", CHECKED_OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Build the HIP library libzkntt.so in-tree with hipcc for gfx950.

Each source compiles to its own object in parallel; the objects link into one
shared library next to this file, which the Python binding loads.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libzkntt.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["api.cpp", "ntt_kernels.hip", "ntt_batch.hip", "microbench.hip",
           "ntt_pass_bls_e3.hip", "ntt_pass_bls_e2.hip", "ntt_pass_bls_e1.hip",
           "ntt_pass_bn_e3.hip", "ntt_pass_bn_e2.hip", "ntt_pass_bn_e1.hip",
           "ntt_pass_b377_e3.hip", "ntt_pass_b377_e2.hip", "ntt_pass_b377_e1.hip",
           "ntt_pass_bls_f64_e2.hip", "msm.hip"]

ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _deps(path: str, seen: set | None = None) -> set:
    """The file and every header it includes with #include "..." (found next
    to it, in csrc/ or in include/), recursively."""
    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    with open(path) as f:
        for m in re.finditer(r'^\s*#\s*include\s+"([^"]+)"', f.read(), re.M):
            for d in (os.path.dirname(path), CSRC, os.path.join(ROOT, "include")):
                cand = os.path.normpath(os.path.join(d, m.group(1)))
                if os.path.exists(cand):
                    _deps(cand, seen)
                    break
    return seen


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    path = os.path.join(CSRC, src)
    if incremental and os.path.exists(obj):
        if os.path.getmtime(obj) >= max(os.path.getmtime(d) for d in _deps(path)):
            return obj
    cmd = [hipcc(), *COMMON, "-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source and link the library.  incremental=True skips
    objects newer than their source and the headers it includes (for
    development; the default always compiles everything)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    sys.exit(0)

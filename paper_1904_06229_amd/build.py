"""Build libperm.so (HIP kernels for gfx950 + the C-ABI runtime) in-tree.

Every source is compiled by hipcc for gfx950 only.  Flags:
  -ffp-contract=off      the error-free transformations (TwoSum, the exact
                         splits of the 0/1 walk) must not be fused into fma;
                         fma is written explicitly where it is wanted.
  -packed-fp32-ops off   no packed FP32 instructions are generated.
No fast-math.  The sources are compiled in parallel, then linked.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libperm.so")
BUILD_DIR = os.path.join(ROOT, "_build")

# (source, extra defines): the walk families are split by size range into two
# translation units each so that they compile in parallel.
SOURCES = [
    ("kern_real.hip", ["-DPERM_HALF=0"]),
    ("kern_real.hip", ["-DPERM_HALF=1"]),
    ("kern_complex.hip", ["-DPERM_HALF=0"]),
    ("kern_complex.hip", ["-DPERM_HALF=1"]),
    ("kern_int01.hip", ["-DPERM_HALF=0"]),
    ("kern_int01.hip", ["-DPERM_HALF=1"]),
    ("kern_mixed.hip", ["-DPERM_CPLX=0", "-DPERM_HALF=0"]),
    ("kern_mixed.hip", ["-DPERM_CPLX=0", "-DPERM_HALF=1"]),
    ("kern_mixed.hip", ["-DPERM_CPLX=1", "-DPERM_HALF=0"]),
    ("kern_mixed.hip", ["-DPERM_CPLX=1", "-DPERM_HALF=1"]),
    ("kern_mixed_stage.hip", []),
    ("kern_band.hip", []),
    ("kern_stage.hip", []),
    ("kern_fused.hip", []),
    ("kern_batched.hip", []),
    ("perm_host.cpp", []),
    ("perm_batched.cpp", []),
    ("perm_mixed.cpp", []),
    ("perm_band.cpp", []),
    ("perm_noalloc.hip", []),
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
]


def _compile(job) -> str:
    src, defines = job
    path = os.path.join(CSRC, src)
    tag = "".join(d.replace("-D", "_").replace("=", "") for d in defines)
    obj = os.path.join(BUILD_DIR, src + tag + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + FLAGS + defines + lang + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s[0]))]
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()

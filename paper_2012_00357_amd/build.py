"""Build libdd.so (HIP, gfx950) from csrc/*.hip with hipcc.

    python -m paper_2012_00357_amd.build        # or build() from Python

Every translation unit is compiled to an object under _build/ in parallel and
linked into paper_2012_00357_amd/libdd.so (in-tree, next to this file).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libdd.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from emitting packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


# Matrix-core scan kernels: inputs are finite, so IEEE mode and NaN semantics
# are off (min reductions need no canonicalisation) and MFMA results stay in
# ordinary VGPRs instead of round-tripping through AGPRs.
FINITE_FLAGS = ["-fno-honor-nans", "-mno-amdgpu-ieee"]
MFMA_FLAGS = FINITE_FLAGS + ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
# The tree walks: the same for their box and ball bounds (queries with
# non-finite coordinates leave the walk before any arithmetic).
FINITE_SOURCES = ("ann.hip",)


def _compile(src: str) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    name = os.path.basename(src)
    extra = MFMA_FLAGS if name.endswith("_mfma.hip") else FINITE_FLAGS if name in FINITE_SOURCES else []
    cmd = [_hipcc(), *HIPCC_FLAGS, *extra, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    sources = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    jobs = min(len(sources), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, sources))
    tmp = OUT + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} from {len(sources)} sources")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Build libttround.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2110_04393_amd.build      # or build() from Python

Every translation unit under csrc/ is compiled for gfx950 only, with packed
FP32 instructions disabled, and linked into one shared library next to this
file.  The library exports only the extern "C" symbols of include/tt_round.h.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libttround.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    "-munsafe-fp-atomics",
    # the small factorisation kernels unroll their step loops completely so
    # that per-thread matrix slices stay in registers
    "-mllvm", "-pragma-unroll-threshold=500000",
]


# One-workgroup factorisation kernels that read and write MFMA accumulators
# with ordinary vector instructions between the products (the blocked
# Cholesky, the eigen finish, the second truncation pass): accumulators in
# VGPRs instead of AGPRs, which saves the copies between the two files.  The
# streaming GEMM and W-chain kernels keep the default (AGPRs as extra room).
PER_FILE = {
    "smallqr.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "tri_eig.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
    "trunc_refine.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    cmd = [HIPCC, *COMMON, *PER_FILE.get(os.path.basename(src), []), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    return obj, warn


def _stale(src):
    """True when the object of src is missing or older than src or any header."""
    obj = os.path.join(BUILD, os.path.basename(src).replace(".hip", ".o"))
    if not os.path.exists(obj):
        return True
    heads = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    heads.append(os.path.join(os.path.dirname(HERE), "include", "tt_round.h"))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(f) > t for f in [src, *heads] if os.path.exists(f))


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source (incremental: only those whose object is stale)
    and link the library."""
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    todo = [s for s in srcs if _stale(s)] if incremental else srcs
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        results = list(ex.map(_compile, todo))
    if verbose:
        for obj, warn in results:
            if warn:
                print(warn, file=sys.stderr)
    objs = [os.path.join(BUILD, os.path.basename(s).replace(".hip", ".o")) for s in srcs]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs,
           "-Wl,--no-undefined", "-Wl,-soname,libttround.so"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))

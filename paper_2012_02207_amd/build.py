"""Builds the gfx950 FMM library ``libfmm_hip.so`` in-tree with hipcc.

Every translation unit is compiled with -ffp-contract=off (the arithmetic that
feeds the acceptance test must round exactly as written; evaluation kernels
ask for fused multiply-adds explicitly) and with packed FP32 instructions
disabled.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfmm_hip.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["api.hip", "tree.hip", "upward.hip", "walk.hip", "m2l.hip", "m2l_hi.hip", "m2l_mixed.hip",
           "local.hip", "adjoint.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-I" + os.path.join(HERE, "..")]


def _headers():
    inc = os.path.join(HERE, "..", "include")
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    return hs + [os.path.join(inc, f) for f in os.listdir(inc) if f.endswith(".h")]


def _compile(src, incremental=False):
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if all(os.path.getmtime(f) < t for f in [os.path.join(CSRC, src)] + _headers()):
            return obj, ""
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False, jobs=8, incremental=False):
    """Compiles every source (incremental=True skips objects newer than their
    source and every header) and links the shared library."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, incremental), SOURCES))
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv)
    print(LIB)

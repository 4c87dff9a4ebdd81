"""Builds libfredec.so (HIP, gfx950) in-tree with hipcc: one object per
source (compiled in parallel), then one shared library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfredec.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["fredec_api.hip", "fredec_tuples_api.hip", "prep.hip", "scan_f64.hip", "rescore.hip", "scan_f32.hip", "scan_f16x3.hip", "tuples.hip", "select.hip",
           "fredec_select_api.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
# Per-source additions.  The tuple Gram kernels and the split-float16 scan keep
# their MFMA accumulators in loop-carried registers; the VGPR form of the MFMA
# lets them stay in the registers the MFMA writes (with the
# accumulation-register form the compiler copies accumulators out and back in
# inside the loops).
_MFMA_VGPR = ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
FILE_FLAGS = {
    "tuples.hip": _MFMA_VGPR,
    "scan_f16x3.hip": _MFMA_VGPR,
}


def _compile(src: str, extra, verbose: bool) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *FILE_FLAGS.get(src, []), *extra, "-I", INCLUDE, "-I", CSRC, "-c",
           os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed compiling {src}")
    return obj


def build(verbose: bool = False, extra=()) -> str:
    """Compile every HIP source into paper_1309_0100_amd/libfredec.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8"))))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        objs = list(pool.map(lambda s: _compile(s, extra, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-fPIC", "-shared", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libfredec.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])

"""Builds libgpz.so (the gfx950 HIP kernels and the C ABI) in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libgpz.so")
SOURCES = ["api.hip", "encode.hip", "decode.hip", "aux.hip", "batch.hip", "generic.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # IEEE arithmetic exactly as written: no contraction, denormals kept
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero", "-fno-fast-math",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


BENCH_LIB = os.path.join(OUT_DIR, "libgpzbench.so")
BENCH_SOURCES = ["membench.hip"]


def build_lib(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libgpz.so and the
    bandwidth probes' libgpzbench.so (always rebuilds)."""
    _link(SOURCES, LIB, verbose)
    _link(BENCH_SOURCES, BENCH_LIB, verbose)
    return LIB


def _link(sources, lib, verbose):
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    for src in sources:
        obj = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
        cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c",
               os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose and r.stderr:
            print(r.stderr)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build_lib(verbose=True))

"""Build libntc.so (all HIP sources, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libntc.so")
SOURCES = ["ntc_api.hip", "ntc_plain.hip", "ntc_mfma.hip", "ntc_backward.hip", "ntc_batched.hip", "ntc_qat.hip",
           "ntc_classify.hip", "ntc_filtered.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-fno-gpu-rdc",
    "-I" + INCLUDE,
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
]


# Matrix-core results in arch VGPRs, where the decode epilogues read them
# directly; the backward (one wavefront per SIMD, 512 registers) keeps its
# gradient accumulators in the accumulation registers instead.
PER_FILE = {s: ["-mllvm", "-amdgpu-mfma-vgpr-form=1"] for s in SOURCES if s != "ntc_backward.hip"}


def _compile(src: str, obj: str, extra, verbose: bool) -> None:
    cmd = [HIPCC] + FLAGS + PER_FILE.get(os.path.basename(src), []) + list(extra or []) + ["-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, extra=None) -> str:
    """Compile every source to an object (in parallel), then link libntc.so."""
    from concurrent.futures import ThreadPoolExecutor

    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    workers = max(1, min(len(srcs), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as ex:
        for f in [ex.submit(_compile, s, o, extra, verbose) for s, o in zip(srcs, objs)]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-fno-gpu-rdc", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])

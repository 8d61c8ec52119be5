"""Build the gfx950 shared library librlqr.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["rlqr_kernels.hip", "rlqr_kernels_mw.hip", "rlqr_scan.hip", "rlqr_api.hip", "rlqr_noalloc.hip", "rlqr_spd.hip", "rlqr_xs.hip", "rlqr_eq.hip", "ripm.hip", "rmlp.hip"]
LIB = os.path.join(HERE, "librlqr.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed float32 arithmetic in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel, one hipcc per file) and link."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = jobs or min(len(SOURCES), max(1, min(os.cpu_count() or 1, 16)))
    objs = [os.path.join(CSRC, src + ".o") for src in SOURCES]

    def compile_one(i):
        cmd = [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(compile_one, i) for i in range(len(SOURCES))]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

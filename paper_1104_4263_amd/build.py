"""Build the HIP shared library libdie_te.so in-tree for gfx950.

Compiles every source under csrc/ with hipcc and links them into
paper_1104_4263_amd/libdie_te.so.  Run as a script or call build().
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libdie_te.so")
SOURCES = ["kernels_fft.hip", "kernels_krylov.hip", "kernels_block.hip", "kernels_gemm.hip", "kernels_unet.hip",
           "scratch.hip", "die_te.cpp", "unet.cpp", "plan.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# The FFT passes fold known-zero padding (x + 0 -> x), which is exact up to the sign of zero.
EXTRA = {"kernels_fft.hip": ["-fno-signed-zeros"]}


def _compile(src: str, obj: str) -> None:
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *EXTRA.get(src, []),
           "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{res.stdout}\n{res.stderr}")


def build(verbose: bool = True) -> str:
    with tempfile.TemporaryDirectory(prefix="die_te_build_") as tmp:
        objs = [os.path.join(tmp, os.path.splitext(s)[0] + ".o") for s in SOURCES]
        with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
            list(ex.map(lambda so: _compile(*so), zip(SOURCES, objs)))
        out_tmp = LIB + ".tmp"
        cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp] + objs + \
            ["-lpthread"]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"linking failed:\n{res.stdout}\n{res.stderr}")
        os.replace(out_tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)

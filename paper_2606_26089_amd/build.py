"""Build libfmdet.so (HIP kernels + C ABI) for gfx950 with hipcc.

Usage: python -m paper_2606_26089_amd.build [--jobs N] [--debug]
The library is written next to this file; object files go to _build/ at the repo root.
"""

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libfmdet.so")

SOURCES = ["gemm_bf16.hip", "gemm_f32.hip", "kernels_misc.hip", "gemm.hip", "attention.hip", "block_bf16.hip",
           "engine.cpp", "server.cpp", "select_noalloc.hip"]
HEADERS = ["common.h", "kernels.h", "engine.h", "engine_impl.h", "gemm_body.h", "gemm_inst.h",
           os.path.join("..", "..", "include", "fmd.h")]

ARCH = "gfx950"
COMMON_FLAGS = [
    f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-variable",
    "-Wno-unused-but-set-variable", "-Wno-unused-function",
    # never let the compiler form packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found: the HIP toolchain (ROCm) is required to build fmdet")


def _compile(src: str, opt: list) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + COMMON_FLAGS + opt
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if r.stderr.strip():
        noise = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if noise:
            sys.stderr.write("\n".join(noise) + "\n")
    return obj


def build(jobs: int | None = None, debug: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    opt = ["-O1", "-g"] if debug else ["-O3"]
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, opt), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--debug", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.debug))


if __name__ == "__main__":
    main()

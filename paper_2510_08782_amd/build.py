"""Build libganmres.so (gfx950) from the HIP sources in csrc/.

Usage: python -m paper_2510_08782_amd.build [--checked]  (or build() from Python).
Each translation unit is compiled in parallel with hipcc, then linked into
paper_2510_08782_amd/_lib/libganmres.so.

--checked builds libganmres_checked.so instead, with GAN_CHECK_TAPS defined:
a gather whose interpolation stencil falls outside the window staged in LDS
poisons that point with NaN (the evaluation then fails with
GANMRES_ENONFINITE) instead of clamping the LDS index.  The binding loads it
when GANMRES_CHECKED=1 is set in the environment.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB = os.path.join(OUT_DIR, "libganmres.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions stay off (compiler-generated v_pk_* f32 forms)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]
LIB_CHECKED = os.path.join(OUT_DIR, "libganmres_checked.so")
SOURCES = ["sl.hip", "spectral.hip", "vec.hip", "runtime.hip", "noalloc.hip"]


def _compile(src: str, checked: bool) -> str:
    bdir = os.path.join(BUILD_DIR, "checked") if checked else BUILD_DIR
    obj = os.path.join(bdir, src + ".o")
    extra = ["-DGAN_CHECK_TAPS"] if checked else []
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    if r.stderr.strip():
        sys.stderr.write(r.stderr)
    return obj


def build(verbose: bool = True, checked: bool = False) -> str:
    lib = LIB_CHECKED if checked else LIB
    os.makedirs(OUT_DIR, exist_ok=True)
    os.makedirs(os.path.join(BUILD_DIR, "checked") if checked else BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(lambda s: _compile(s, checked), SOURCES))
    tmp = lib + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(checked="--checked" in sys.argv[1:])

"""Build libimpconv.so for gfx950 with hipcc (one object per translation unit,
compiled in parallel, linked into the package directory)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libimpconv.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
EXTRA = os.environ.get("IMPCONV_CXXFLAGS", "").split()
ARCH = "gfx950"
# -packed-fp32-ops: keep the compiler from emitting packed FP32 arithmetic
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-variable", "-Wno-unused-but-set-variable",
         "-I", os.path.join(HERE, "..", "include")]
SOURCES = ["k_row_queue.hip", "k_row_complex.hip", "k_row_comp.hip", "k_row_herm.hip", "k_row_pq.hip", "k_col_pad.hip", "k_col_comp.hip", "k_col_cen.hip", "k_col_ter.hip",
           "k_col_fft.hip", "k_col_fs.hip", "k_misc.hip", "twiddle.hip", "multid.hip",
           "ragged.hip", "schedule.hip", "plan.hip", "noalloc.hip", "abi.hip"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *EXTRA, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int | None = None, out: str | None = None, build_dir: str | None = None) -> str:
    global BUILD
    if build_dir:
        BUILD = build_dir
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else None))

"""Build liblrigw.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "liblrigw.so")
# stand-alone calibration program: the sustained dense FP16 matrix-core rate
RATE_SRC = "mfma_rate.hip"
RATE_BIN = os.path.join(HERE, "mfma_rate")
SOURCES = ["api.hip", "k_grid.hip", "k_lri.hip", "k_build.hip", "k_chi0.hip", "k_sigma.hip", "k_dense.hip",
           "k_screen.hip", "k_qp.hip", "k_surrogate.hip", "k_batch.hip", "k_exchange.hip", "k_fit.hip",
           "k_contour.hip"]
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall", "-Wno-unused-result",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]


def _hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    return p


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _build_rate() -> str:
    tmp = RATE_BIN + ".tmp"
    cmd = [_hipcc(), *FLAGS, os.path.join(CSRC, RATE_SRC), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {RATE_SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, RATE_BIN)
    return RATE_BIN


def build(jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(8, len(SOURCES))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        rate = ex.submit(_build_rate)
        objs = list(ex.map(_compile, SOURCES))
        rate.result()
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
    sys.exit(0)

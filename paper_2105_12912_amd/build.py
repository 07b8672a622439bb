"""Build the HIP C-ABI library ``libebc.so`` for gfx950 (in-tree).

Every HIP source is compiled with hipcc for ``--offload-arch=gfx950`` with
floating-point contraction off (bit-exact prequantisation and dequantisation)
and packed-FP32 instructions disabled, then linked into one shared library
next to this file.  Usage: ``python -m paper_2105_12912_amd.build``.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libebc.so")
ARCH = os.environ.get("EBC_OFFLOAD_ARCH", "gfx950")

SOURCES = [
    "k_quant.hip",
    "k_scan.hip",
    "k_codebook.hip",
    "k_huffman.hip",
    "k_rle.hip",
    "k_outlier.hip",
    "k_recon.hip",
    "k_archive.hip",
    "k_estimate.hip",
    "noalloc.hip",
    "capi.cpp",  # host code only
]

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ROCM_INCLUDE = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "include")
CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "c++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
               "-I", ROCM_INCLUDE, "-I", INCLUDE,
               "-c", os.path.join(CSRC, src), "-o", obj]
    else:
        cmd = [HIPCC, *CFLAGS, "-I", INCLUDE, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l
                     and "not a recognized feature" not in l)
    if warn.strip() and os.environ.get("EBC_BUILD_VERBOSE"):
        print(warn, file=sys.stderr)
    return obj


def build(jobs: int | None = None) -> str:
    """Compile every source and link ``libebc.so``; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 16)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

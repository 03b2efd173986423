"""Builds libchase_mi355x.so (the HIP path) in-tree for gfx950.

Every HIP/C++ source under csrc/ is compiled by hipcc to an object in
_build/ and linked into one shared library next to this file.  Packed FP32
instructions are disabled on purpose (-packed-fp32-ops).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libchase_mi355x.so")
SYNTH_LIB = os.path.join(HERE, "libchase_synth.so")

ARCH = os.environ.get("CHASE_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-result"]

SOURCES = ["k_filter.hip", "k_filter_wide.hip", "k_filter32.hip", "k_filter_fused.hip",
           "k_blas.hip", "k_dense.hip", "k_ingest.hip", "control.cpp", "solver.cpp", "capi.cpp",
           "server.cpp"]
# Input generators live in a library of their own: they are not the solver.
SYNTH_SOURCES = ["synth_dev.hip"]


# MFMA register form per source: the VGPR form keeps the filter tiles'
# accumulators in place through their k loops.
VGPR_FORM = ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]
EXTRA = {"k_filter.hip": VGPR_FORM, "k_filter_wide.hip": VGPR_FORM, "k_filter32.hip": VGPR_FORM,
         "k_blas.hip": VGPR_FORM, "k_dense.hip": VGPR_FORM, "k_filter_fused.hip": VGPR_FORM}


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC, *FLAGS, *EXTRA.get(src, []), *lang, "-c", os.path.join(CSRC, src),
           "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def _link(objs, out, verbose):
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES + SYNTH_SOURCES))
    _link(objs[:len(SOURCES)], LIB, verbose)
    _link(objs[len(SOURCES):], SYNTH_LIB, verbose)
    return LIB


def clean() -> None:
    shutil.rmtree(BUILD, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

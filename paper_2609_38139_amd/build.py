"""Builds the HIP library ``liblaim.so`` in this directory for gfx950.

Every HIP source is compiled with hipcc for gfx950 only, without FP
contraction or fast-math (the decoder's integer decisions come from FP32
messages, which must round exactly as written) and without packed-FP32
instruction selection; the objects are linked into one shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "liblaim.so")
SOURCES = ["laim_kernels.hip", "laim_stream.hip", "laim_ctm.hip", "laim_bitcentric.hip", "laim_host.cpp",
           "laim_batch.cpp", "laim_static.hip", "laim_online.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    # No value on the decoder's path is ever NaN; with IEEE mode off the
    # min/max instructions need no canonicalising copies of their inputs.
    "-fno-honor-nans", "-mno-amdgpu-ieee",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj


# Measurement helpers of the benchmark (VALU and LDS probes), linked into a
# library of their own: they are not part of the decoder.
PROBE_SOURCES = ["laim_probe.hip"]
PROBE_LIB = os.path.join(HERE, "liblaim_probe.so")


def _link(objs, out):
    tmp = out + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile every source (always) and link ``liblaim.so`` and the
    benchmark's ``liblaim_probe.so``."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES) + len(PROBE_SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, SOURCES + PROBE_SOURCES))
    _link(objs[:len(SOURCES)], LIB)
    _link(objs[len(SOURCES):], PROBE_LIB)
    if verbose:
        print(f"built {LIB} and {PROBE_LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

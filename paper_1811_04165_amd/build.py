"""Builds libamber.so (HIP for gfx950) in-tree with hipcc.

Each translation unit under csrc/ is compiled to an object in _build/ and
linked into paper_1811_04165_amd/libamber.so.  Run as a script or call
build().
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libamber.so")
ARCH = os.environ.get("AMBER_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE, "-I" + CSRC, "-Wall", "-Wno-unused-result",
]


# Per-file flags.  dedisperse.hip: its channel loop branches on wave-uniform
# conditions only; without this the structurizer turns each 4-way branch into
# a chain of flow variables and register copies.
EXTRA = {"dedisperse.hip": ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]}


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + EXTRA.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


PEAKS_SRC = os.path.join(PKG, "peaks", "peaks.hip")
PEAKS_LIB = os.path.join(PKG, "libamber_peaks.so")


def build_peaks(verbose: bool = False) -> str:
    """The microbenchmarks behind the roofline peaks (a library of their own,
    loaded only by the benchmark's peak measurement)."""
    tmp = PEAKS_LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "-x", "hip"] + COMMON + ["-shared", "-o", tmp, PEAKS_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (PEAKS_SRC, r.stdout, r.stderr))
    os.replace(tmp, PEAKS_LIB)
    if verbose:
        print("built", PEAKS_LIB)
    return PEAKS_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = min(len(srcs), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    build_peaks(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

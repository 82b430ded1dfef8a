"""Builds libappga.so for gfx950 with hipcc (in-tree, next to this file).

Usage: python -m paper_2409_13344_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libappga.so")
SOURCES = ["kernels.hip", "appga_api.cpp", "server.cpp", "tune.cpp"]
ARCH = os.environ.get("APPGA_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # IEEE FP32 division and square root in device code, no fast-math contractions across ops
    "-fhip-fp32-correctly-rounded-divide-sqrt", "-ffp-contract=on",
    "-Wall", "-Wno-unused-result",
]


def _obj(src: str, outdir: str) -> str:
    return os.path.join(outdir, os.path.splitext(src)[0] + ".o")


def build(verbose: bool = False) -> str:
    outdir = os.path.join(HERE, "_build")
    os.makedirs(outdir, exist_ok=True)

    def compile_one(src):
        path = os.path.join(CSRC, src)
        cmd = ["hipcc", *COMMON, "-x", "hip", "-c", path, "-o", _obj(src, outdir)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
        return r.stderr

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        logs = list(ex.map(compile_one, SOURCES))
    if verbose:
        for lg in logs:
            if lg.strip():
                print(lg)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *[_obj(s, outdir) for s in SOURCES], "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

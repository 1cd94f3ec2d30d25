"""Builds libckkt.so (host analysis + HIP kernels for gfx950) in-tree.

Usage:  python -m paper_2405_14236_amd.build_lib   (or call build()).
Always recompiles; objects go to ``paper_2405_14236_amd/_build``.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libckkt.so")
ARCH = "gfx950"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
HIP_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]
HOST_ONLY = ["analysis.cpp", "ordering.cpp", "hostref.cpp"]
HIP_SRCS = ["kernels.hip", "kernels_mlp.hip", "symbolic.hip", "ckkt.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for s in HOST_ONLY:
        o = os.path.join(BUILD, s + ".o")
        jobs.append((["g++"] + COMMON + ["-c", os.path.join(CSRC, s), "-o", o], o))
    for s in HIP_SRCS:
        o = os.path.join(BUILD, s + ".o")
        extra = ["-x", "hip"] if s.endswith(".cpp") else []
        jobs.append(([HIPCC] + COMMON + HIP_FLAGS + extra + ["-c", os.path.join(CSRC, s), "-o", o], o))
    with ThreadPoolExecutor(max_workers=4) as ex:
        for r in ex.map(lambda j: _run(j[0]), jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + [o for _, o in jobs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

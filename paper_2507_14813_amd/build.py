"""Build ``libmayura.so`` (HIP kernels for gfx950 + host code + C ABI) in-tree.

Run as ``python -m paper_2507_14813_amd.build``.  Cross-compiles without a GPU.
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libmayura.so")
BUILD_DIR = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROCM_INC = os.path.join(os.path.dirname(os.path.dirname(HIPCC)), "include")
ARCH = "gfx950"

# packed FP32 VALU ops stay off in every HIP compile
NO_PK_FP32 = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n%s\n%s" % (" ".join(cmd), r.stdout))
    return out


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for name in ("comine.hip", "sched.hip"):
        obj = os.path.join(BUILD_DIR, name + ".o")
        out = _run([HIPCC, "-x", "hip", "--offload-arch=" + ARCH, *COMMON, *NO_PK_FP32,
                    "-c", os.path.join(CSRC, name), "-o", obj])
        if verbose and out:
            print(out)
        objs.append(obj)
    for name in ("host.cpp",):   # host-only C++ (HIP runtime API, no device code)
        obj = os.path.join(BUILD_DIR, name + ".o")
        out = _run([HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, *COMMON, "-c",
                    os.path.join(CSRC, name), "-o", obj])
        if verbose and out:
            print(out)
        objs.append(obj)
    tmp = OUT + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

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


# the search kernels: one file per (tree depth, time width), largest first
HIP_SOURCES = tuple("search_d%d_t%d.hip" % (d, t) for d in (5, 4, 3, 2, 1) for t in (32, 64)) + \
    ("comine.hip", "sched.hip")


def _compile(name):
    obj = os.path.join(BUILD_DIR, name + ".o")
    if name.endswith(".hip"):
        cmd = [HIPCC, "-x", "hip", "--offload-arch=" + ARCH, *COMMON, *NO_PK_FP32]
    else:   # host-only C++ (HIP runtime API, no device code)
        cmd = [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INC, *COMMON]
    return obj, _run(cmd + ["-c", os.path.join(CSRC, name), "-o", obj])


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel: one process per file, the tree
    depths in separate files) and link libmayura.so."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD_DIR, exist_ok=True)
    names = list(HIP_SOURCES) + ["host.cpp", "cpu.cpp"]
    jobs = jobs or min(len(names), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, names))
    objs = []
    for obj, out in results:
        if verbose and out:
            print(out)
        objs.append(obj)
    tmp = OUT + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-ldl", "-lpthread", "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

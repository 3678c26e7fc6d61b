"""Build the HIP library ``libwh.so`` in-tree for gfx950.

    python -m paper_2504_03074_amd.build

Compiles every source under ``csrc/`` with hipcc for the MI355X (gfx950).
Packed FP32 instructions are disabled for device code.
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libwh.so")
ARCH = "gfx950"

SOURCES = ["wh_block_f64_p4.hip", "wh_block_f32_p4.hip", "wh_block_f64_p2.hip", "wh_block_f32_p2.hip",
           "wh_block3d_f64_p4.hip", "wh_block3d_f32_p4.hip", "wh_block3d_f64_p2.hip", "wh_block3d_f32_p2.hip",
           "wh_kernels.hip", "wh_mg.hip", "wh_block.hip", "wh_noalloc.hip", "wh_api.cpp"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-fvisibility=hidden",
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False, jobs: int = 0) -> str:
    jobs = jobs or max(1, min(len(SOURCES), os.cpu_count() or 4))
    objs = []
    procs = []
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        cmd = [hipcc()] + [f for f in FLAGS if f != "-shared"] + ["-I", INCLUDE, "-I", CSRC, "-c", path, "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-Wall", "-fvisibility=hidden", f"--offload-arch={ARCH}",
                   "-I", INCLUDE, "-I", CSRC, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        if len(procs) >= jobs:
            if procs.pop(0).wait() != 0:
                raise RuntimeError("hipcc failed")
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    link = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Build libat.so (HIP, gfx950) and the CPU emulation library of its kernels.

    python -m paper_2204_01133_amd.build

libat.so: hipcc --offload-arch=gfx950, one object per kernel kind compiled in
parallel, linked into a shared library with the C ABI of include/at.h.
libat_emu.so: the same tile code compiled for the host with bounds checks
(test infrastructure; the product never loads it).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "libat.so")
EMU = os.path.join(BUILD, "libat_emu.so")

HIP_SOURCES = ["at_api.hip", "at_k_adr.hip", "at_k_adr32.hip", "at_k_rns.hip", "at_k_rns32.hip", "at_k_wscal.hip", "at_k_eul.hip",
               "at_k_reul.hip"]
HOST_SOURCES = ["at_plan.cpp"]

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["-std=c++17", "-O3", "--offload-arch=gfx950", "-fPIC", "-ffp-contract=on",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build_lib(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs, cmds = [], []
    for src in HIP_SOURCES + HOST_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = [] if src.endswith(".hip") else ["-x", "c++"]
        cmds.append([HIPCC] + HIP_FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(_run, cmds))
    tmp = LIB + f".tmp{os.getpid()}"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


def build_emu() -> str:
    os.makedirs(BUILD, exist_ok=True)
    tmp = EMU + f".tmp{os.getpid()}"
    _run(["g++", "-std=c++17", "-O1", "-fPIC", "-shared", "-Wall", "-Wno-unused-variable",
          "-Wno-maybe-uninitialized", "-o", tmp, os.path.join(CSRC, "at_emu.cpp"),
          os.path.join(CSRC, "at_plan.cpp")])
    os.replace(tmp, EMU)
    return EMU


def build(jobs: int = 8) -> None:
    with cf.ThreadPoolExecutor(max_workers=2) as ex:
        f1 = ex.submit(build_lib, jobs)
        f2 = ex.submit(build_emu)
        f1.result()
        f2.result()


if __name__ == "__main__":
    build(int(sys.argv[1]) if len(sys.argv) > 1 else 8)
    print(LIB)
    print(EMU)

"""Build libat.so (HIP, gfx950) and the CPU emulation library of its kernels.

    python -m paper_2204_01133_amd.build [JOBS] [--define NAME=VALUE ...] [--lib-only]

AT_BUILD_DIR (environment) puts the build in another folder (default: _build beside
this file); the library loader reads the same variable, so that a build with other
compile-time options (--define, e.g. AT_WENO_DPP=1) can be run side by side.

libat.so: hipcc --offload-arch=gfx950, one object per kernel kind compiled in
parallel, linked into a shared library with the C ABI of include/at.h.
libat_emu.so: the same tile code compiled for the host with bounds checks
(test infrastructure; the product never loads it).
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.environ.get("AT_BUILD_DIR") or os.path.join(HERE, "_build")
LIB = os.path.join(BUILD, "libat.so")
EMU = os.path.join(BUILD, "libat_emu.so")

HIP_SOURCES = ["at_api.hip", "at_k_adr.hip", "at_k_adr32.hip", "at_k_rns.hip", "at_k_rns32.hip", "at_k_wscal.hip", "at_k_eul.hip",
               "at_k_reul.hip"]
HOST_SOURCES = ["at_plan.cpp"]

STAMP = os.path.join(BUILD, "libat.stamp")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")


def source_files():
    """Every source libat.so is built from (kernels, planner, C ABI header)."""
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                   if f.endswith((".hip", ".hpp", ".cpp", ".h")))
    return files + [os.path.join(INCLUDE, "at.h")]


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of the sources, written beside the library when it
    is built and compared when it is loaded, so that a stale build is refused."""
    h = hashlib.sha256()
    for f in source_files():
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]
HIP_FLAGS = ["-std=c++17", "-O3", "--offload-arch=gfx950", "-fPIC", "-ffp-contract=on",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    return out


def build_lib(jobs: int = 8, defines=()) -> str:
    os.makedirs(BUILD, exist_ok=True)
    stamp = source_hash()
    objs, cmds = [], []
    dflags = ["-D" + d for d in defines]
    for src in HIP_SOURCES + HOST_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        lang = [] if src.endswith(".hip") else ["-x", "c++"]
        cmds.append([HIPCC] + HIP_FLAGS + dflags + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(_run, cmds))
    tmp = LIB + f".tmp{os.getpid()}"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    with open(STAMP + ".tmp", "w") as fh:
        fh.write(stamp + "\n")
    os.replace(STAMP + ".tmp", STAMP)
    return LIB


def build_emu() -> str:
    os.makedirs(BUILD, exist_ok=True)
    tmp = EMU + f".tmp{os.getpid()}"
    _run(["g++", "-std=c++17", "-O1", "-fPIC", "-shared", "-Wall", "-Wno-unused-variable",
          "-Wno-maybe-uninitialized", "-o", tmp, os.path.join(CSRC, "at_emu.cpp"),
          os.path.join(CSRC, "at_plan.cpp")])
    os.replace(tmp, EMU)
    return EMU


def build(jobs: int = 8, defines=(), lib_only: bool = False) -> None:
    with cf.ThreadPoolExecutor(max_workers=2) as ex:
        f1 = ex.submit(build_lib, jobs, defines)
        f2 = None if lib_only else ex.submit(build_emu)
        f1.result()
        if f2 is not None:
            f2.result()


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("jobs", nargs="?", type=int, default=8)
    ap.add_argument("--define", action="append", default=[], help="NAME=VALUE for the HIP compile")
    ap.add_argument("--lib-only", action="store_true", help="skip the CPU emulation library")
    a = ap.parse_args()
    build(a.jobs, a.define, a.lib_only)
    print(LIB)
    if not a.lib_only:
        print(EMU)

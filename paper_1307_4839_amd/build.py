"""Build the HIP library in-tree with hipcc for gfx950.

``python -m paper_1307_4839_amd.build`` compiles ``csrc/*.hip`` into
``paper_1307_4839_amd/libswe_mi355x.so``.  Cross-compiles without a GPU.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libswe_mi355x.so")
SOURCES = ["swe_step.hip", "swe_batch.hip", "swe_adjoint.hip", "swe_flowdir.hip"]
HEADERS = ["swe_device.h", "swe_host.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # formulas are evaluated as written: no contraction into FMAs
    "-ffp-contract=off",
    # never emit packed FP32 arithmetic
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# the files the stage kernels of the single-simulation library are built from
STAGE_SOURCES = [os.path.join(CSRC, f) for f in ("swe_device.h", "swe_host.h", "swe_step.hip")] + [
    os.path.join(INCLUDE, "swe.h")]


# the files the flow-direction kernel is built from
FLOWDIR_SOURCES = [os.path.join(CSRC, "swe_flowdir.hip"), os.path.join(INCLUDE, "swe_flowdir.h"),
                   os.path.join(INCLUDE, "swe.h")]


def source_hash(paths=None) -> str:
    """Short hash of kernel sources (names and contents; the stage kernels'
    by default), which ties measured counters to a kernel version."""
    import hashlib
    h = hashlib.sha256()
    for path in (STAGE_SOURCES if paths is None else paths):
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = True) -> str:
    """Compile each source to an object in parallel (separate translation
    units, as one hipcc line over all of them would), then link."""
    from concurrent.futures import ThreadPoolExecutor
    tag = f".tmp{os.getpid()}"
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    jobs = []
    for s in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(s)[0] + tag + ".o")
        jobs.append((obj, [hipcc(), *compile_flags, "-I", INCLUDE, "-c",
                           os.path.join(CSRC, s), "-o", obj]))

    def run(job):
        if verbose:
            print(" ".join(job[1]), flush=True)
        subprocess.check_call(job[1])
        return job[0]

    workers = max(1, min(len(jobs), os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(run, jobs))
    tmp = LIB + tag
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp,
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)

"""Builds liblbm.so (the HIP library behind include/lbm.h) in-tree for gfx950,
and liblbm_cpu.so (the paper's sequential CPU algorithms behind
include/lbm_cpu.h, host context).

    python -m paper_2208_05429_amd.build [--resource-usage]

Every source under csrc/ is compiled by hipcc to an object in _build/ (in
parallel) and linked into paper_2208_05429_amd/liblbm.so.  Packed FP32 vector
instructions are disabled for all device code.  host/lbm_cpu.cpp is compiled by
g++ (-O3, no fast-math) into paper_2208_05429_amd/liblbm_cpu.so.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build", "lbm")
LIB = os.path.join(HERE, "liblbm.so")
CPU_SRC = os.path.join(HERE, "host", "lbm_cpu.cpp")
CPU_LIB = os.path.join(HERE, "liblbm_cpu.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function", "-ffp-contract=off",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          f"-I{os.path.join(os.path.dirname(HERE), 'include')}"]


# the sources the FP32 D3Q19 marching kernels and their launch configuration
# are built from (the kernels' code and the host's choice of shape, segments
# and grid); stored counters of those kernels carry this digest
MARCH_SOURCES = ("d3q19.hpp", "lattices.hpp", "lbm_internal.hpp", "march.hpp", "march_pr.hpp", "march_dispatch.hpp",
                 "march_f32.hip", "march_plan.hpp", "march_plan.cpp")


def source_digest(names=MARCH_SOURCES) -> str:
    """Hash of the given csrc sources (default: those of the marching kernels):
    a stored measurement of a kernel is valid while this is unchanged."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(names):
        h.update(name.encode())
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


# Extra hipcc flags per source.  The FP64 marching kernel that loads two
# planes ahead runs its plane iteration as two inlined bodies (one per load
# buffer); at the default inlining threshold the second stays a call and the
# load buffers go to scratch memory.
EXTRA_FLAGS = {"march_f64.hip": ["-mllvm", "-inline-threshold=100000"]}


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src, resource_usage):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + COMMON + EXTRA_FLAGS.get(os.path.basename(src), []) + ["-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd[1:1] = ["-x", "hip"]
    if resource_usage:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    p = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, p.returncode, p.stdout + p.stderr


def build_cpu() -> str:
    """The host library of the paper's CPU algorithms (g++, one thread)."""
    tmp = CPU_LIB + ".tmp"
    cmd = [os.environ.get("CXX", "g++"), "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
           f"-I{os.path.join(os.path.dirname(HERE), 'include')}", "-o", tmp, CPU_SRC]
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"g++ failed on lbm_cpu.cpp:\n{p.stdout}{p.stderr}")
    os.replace(tmp, CPU_LIB)
    return CPU_LIB


def build(resource_usage: bool = False, jobs: int | None = None, verbose: bool = False) -> str:
    build_cpu()
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    objs, logs = [], []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for src, obj, rc, out in ex.map(lambda s: _compile(s, resource_usage), srcs):
            if rc != 0:
                raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{out}")
            objs.append(obj)
            if out.strip():
                logs.append(f"== {os.path.basename(src)}\n{out}")
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"link failed:\n{p.stdout}{p.stderr}")
    os.replace(tmp, LIB)
    if resource_usage or verbose:
        with open(os.path.join(BUILD, "build.log"), "w") as fh:
            fh.write("\n".join(logs))
        if verbose:
            sys.stdout.write("\n".join(logs))
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--resource-usage", action="store_true")
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.resource_usage, verbose=a.verbose))

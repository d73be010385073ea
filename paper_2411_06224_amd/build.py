"""Builds libmaspcg.so (HIP for gfx950 + host C++) in-tree."""

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmaspcg.so")

HIP_SOURCES = ["spmv.hip", "vectors.hip", "mas.hip", "assemble.hip", "hierarchy.hip", "morton.hip", "abd.hip", "replan.hip", "abi.cpp"]
HOST_SOURCES = ["planner.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang",
    "-target-feature",
    "-Xclang",
    "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-command-line-argument",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(jobs=5, csrc=CSRC, out_dir=OUT, lib=LIB, extra_flags=()):
    """Compile every source and link libmaspcg.so; always rebuilds."""
    os.makedirs(out_dir, exist_ok=True)
    cmds = []
    objs = []
    for f in HIP_SOURCES:
        o = os.path.join(out_dir, f + ".o")
        cmds.append([HIPCC, *DEVICE_FLAGS, *extra_flags, "-x", "hip", "-c", os.path.join(csrc, f), "-o", o])
        objs.append(o)
    for f in HOST_SOURCES:
        o = os.path.join(out_dir, f + ".o")
        cmds.append(["g++", *HOST_FLAGS, "-c", os.path.join(csrc, f), "-o", o])
        objs.append(o)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_run, cmds))
    tmp = lib + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,--no-undefined", "-o", tmp, *objs, "-L/opt/rocm/lib", "-lamdhip64"])
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build())

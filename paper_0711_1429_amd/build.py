"""Build libtc.so (HIP for gfx950) in-tree: ``python -m paper_0711_1429_amd.build``."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtc.so")
SOURCES = ["host_setup.cpp", "kernels.hip", "tc_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


# the compiler's per-kernel resource report of kernels.hip (registers,
# spills, scratch, occupancy), kept beside the objects for the tests
RESOURCES = os.path.join(HERE, "_build", "kernels.resource-usage.txt")


def build(verbose=True):
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, src + ".o")
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        report = src == "kernels.hip"
        if report:
            cmd += ["-Rpass-analysis=kernel-resource-usage", "-fno-caret-diagnostics"]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, stderr=subprocess.PIPE, text=True)
        remarks = [l for l in res.stderr.splitlines() if "kernel-resource-usage" in l]
        other = [l for l in res.stderr.splitlines() if "kernel-resource-usage" not in l]
        if other:
            print("\n".join(other), file=sys.stderr, flush=True)
        if res.returncode != 0:
            raise subprocess.CalledProcessError(res.returncode, cmd)
        if report:
            with open(RESOURCES, "w") as f:
                f.write("\n".join(remarks) + "\n")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-fPIC", *objs, "-o", tmp,
           "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)

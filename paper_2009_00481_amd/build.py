"""Build libbddmp.so in-tree: host C++ with g++, HIP kernels with hipcc for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libbddmp.so")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("BDDMP_ARCH", "gfx950")

HOST_SOURCES = ["primal.cpp", "builder.cpp", "plan.cpp", "capi.cpp"]
HIP_SOURCES = ["kernels.hip", "smooth.hip", "split.hip", "solver.hip"]
# packed fp32 instructions stay off in every device build
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-Wall", "-Wno-unused-result"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r


HOST_ONLY_SOURCES = ["primal.cpp", "builder.cpp", "plan.cpp", "capi.cpp", "solver_host_only.cpp"]
HOST_ONLY_LIB = os.path.join(HERE, "libbddmp_host_san.so")
# the host-only test build under the CPU sanitizers (run with libasan preloaded; see README)
SANITIZE_FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build_host_only(verbose: bool = False) -> str:
    """The host half of the library (builder, planner, primal search, C-ABI checks) with the solver
    calls stubbed to fail with BDDMP_DEVICE, built with AddressSanitizer and UBSan for the CPU tests."""
    objs = []
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", INCLUDE, "-I", CSRC]
    for src in HOST_ONLY_SOURCES:
        o = os.path.join(OBJ, "san_" + src + ".o")
        _run(["g++", *HOST_FLAGS, *SANITIZE_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = HOST_ONLY_LIB + ".tmp"
    _run(["g++", "-shared", "-fPIC", *SANITIZE_FLAGS, *objs, "-o", tmp])
    os.replace(tmp, HOST_ONLY_LIB)
    if verbose:
        print("built", HOST_ONLY_LIB)
    return HOST_ONLY_LIB


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    objs = []
    inc = ["-I", INCLUDE, "-I", CSRC]
    for src in HOST_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        _run(["g++", *HOST_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for src in HIP_SOURCES:
        o = os.path.join(OBJ, src + ".o")
        _run([HIPCC, *HIP_FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    if "--host-only-sanitized" in sys.argv:
        build_host_only(verbose=True)
    else:
        build(verbose=True)

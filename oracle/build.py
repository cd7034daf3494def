"""Compile the CPU oracle (plain C) into two shared objects: fp64 and its fp32 mirror.

Test infrastructure: only tests, the smoke check and the benchmark's CPU-baseline leg use it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bddmp_oracle.c")
# BDDMP_SANITIZE=1: the oracle built with AddressSanitizer and UBSan (run with libasan preloaded)
SANITIZE = os.environ.get("BDDMP_SANITIZE") == "1"
_SUFFIX = "_san" if SANITIZE else ""
TARGETS = {"f64": os.path.join(HERE, f"liboracle_f64{_SUFFIX}.so"), "f32": os.path.join(HERE, f"liboracle_f32{_SUFFIX}.so")}
SANITIZE_FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build(force: bool = True) -> dict:
    for prec, out in TARGETS.items():
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
               "-Wall", "-Wextra", "-Wno-unused-parameter", SRC, "-o", out + ".tmp", "-lm"]
        if SANITIZE:
            cmd[1:1] = SANITIZE_FLAGS
        if prec == "f32":
            cmd.insert(1, "-DORC_REAL_FLOAT")
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
    return TARGETS


if __name__ == "__main__":
    build(force="--if-stale" not in sys.argv)
    print("built", ", ".join(TARGETS.values()))

"""Build the CPU oracle shared library with gcc (test infrastructure).

Generic x86-64 code (no -march=native: the library is built in one place and
may run on another host), FP64 with -ffp-contract=off, OpenMP for the
red-black sweeps used by the CPU baseline.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "subsurf4d_oracle.c")
LIB = os.path.join(HERE, "liboracle_subsurf4d.so")


def build_oracle(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_oracle_native(out_dir: str) -> str:
    """A copy of the oracle compiled for the host it runs on (-march=native),
    for timing the CPU baseline there; the tests use the generic build."""
    os.makedirs(out_dir, exist_ok=True)
    out = os.path.join(out_dir, "liboracle_subsurf4d_native.so")
    cmd = ["gcc", "-O3", "-march=native", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-o", out, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build_oracle())

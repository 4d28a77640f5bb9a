"""Build the oracle's shared library (test infrastructure only).

``build()``: the parity build, ``g++ -O2 -ffp-contract=off`` so that no
multiply-add is fused behind the reader's back; the tests, the smoke check and
the CPU-baseline leg of the benchmark load it.

``build_timing(path)``: the same source, untouched, compiled
``-O3 -march=native`` for the host it runs on; the benchmark times it next to
the parity build (compiler flags alone move a serial CPU code by several
times, as the paper's gcc/icc comparison shows), and never uses it for parity.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emma_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-o", LIB, SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


def build_timing(path, verbose=False):
    """Timing-only build for the machine that runs it (not portable: build it
    where it runs)."""
    cmd = ["g++", "-std=c++17", "-O3", "-march=native", "-fPIC", "-shared", "-o", path, SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return path


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the oracle's shared library (TEST INFRASTRUCTURE).

The parity build uses ``-O2 -ffp-contract=off`` so that no fused multiply-add
changes the rounding of the plain definition. The timing build (the CPU
baseline the GPU path is reported beside) is the same source compiled
``-O3 -march=native -fopenmp`` for the host it runs on.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pkh_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(force=True):
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wall", "-Wno-unused-function", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def build_timing(out_path):
    """The timing build at out_path, tuned for this host's CPU (so it is
    compiled where it runs)."""
    tmp = out_path + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c11",
           "-Wno-unused-function", SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out_path)
    return out_path


if __name__ == "__main__":
    print(build())

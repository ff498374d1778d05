"""Build the CPU oracle (test infrastructure) as a shared library with gcc.

Plain C, -O2, no fast-math and no floating-point contraction, so every
operation is a separately rounded IEEE binary64 operation."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    srcs = [os.path.join(HERE, f) for f in ("dsmc_oracle.c", "dig_oracle.c")]
    cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB + ".tmp", *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

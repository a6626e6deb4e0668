"""Build the CPU oracle shared library (test infrastructure only): the
plain triple sums (sho_oracle.c) and the factorised CPU path that the
benchmark times beside them (sho_factorised.c).

gcc -O2 -fopenmp -ffp-contract=off: no FMA contraction, so the support
membership test is evaluated in the operation order the source states.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sho_oracle.c")
# the factorised CPU path of the benchmark's baseline (pinned to the oracle)
SRC_FACT = os.path.join(HERE, "sho_factorised.c")
LIB = os.path.join(HERE, "libsho_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-shared", "-fPIC", "-o", LIB + ".tmp",
           SRC, SRC_FACT, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)

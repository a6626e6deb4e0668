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


# Sanitizer build (libsho_oracle_asan.so, for the CPU test suite run with
# clang's sanitizer runtime preloaded): clang with AddressSanitizer and
# UndefinedBehaviorSanitizer, OpenMP from the same toolchain.
LIB_ASAN = os.path.join(HERE, "libsho_oracle_asan.so")
CLANG = "/opt/rocm/llvm/bin/clang"


def build(verbose: bool = False, sanitize: bool = False) -> str:
    lib = LIB_ASAN if sanitize else LIB
    cc = [CLANG, "-fsanitize=address", "-fsanitize=undefined",
          "-fno-sanitize-recover=undefined", "-shared-libsan", "-g",
          "-Wl,-rpath,/opt/rocm/llvm/lib"] if sanitize else ["gcc"]
    cmd = cc + ["-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp",
                "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
                "-Wno-unused-parameter", "-shared", "-fPIC", "-o", lib + ".tmp",
                SRC, SRC_FACT, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)

"""Build libsho.so in-tree for gfx950 (hipcc cross-compiles without a GPU).

Objects:
  sho_plan.cpp     host geometry, g++ -ffp-contract=off (the support membership
                   test must be evaluated in the documented operation order)
  sho_setup.cpp    set-up side of the basis (host only), g++
  sho_api.cpp      C ABI layer (host HIP runtime calls)
  sho_server.cpp   request server: admission under a byte budget, streams
  sho_kernels.hip  gfx950 kernels
  sho_kernels_f32.hip  single-precision projection and expansion kernels
"""
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsho.so")
ARCH = os.environ.get("SHO_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result", "-I", INCLUDE, "-I", CSRC]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off",
              "-fno-fast-math", "-Wall", "-Wextra", "-I", INCLUDE, "-I", CSRC]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


# Host-code sanitizer build (libsho_asan.so, for the CPU test suite): the
# host sources with clang's AddressSanitizer and UndefinedBehaviorSanitizer,
# the HIP sources with the same on their host side only (-Xarch_host), linked
# against clang's shared sanitizer runtime, which the test process preloads.
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined"]
LIB_ASAN = os.path.join(PKG, "libsho_asan.so")


def build(verbose: bool = False, jobs: int = 3, sanitize: bool = False) -> str:
    """Compile every source and link libsho.so (always rebuilds); with
    sanitize, the host-sanitized libsho_asan.so instead."""
    bdir = os.path.join(BUILD, "asan") if sanitize else BUILD
    os.makedirs(bdir, exist_ok=True)
    t0 = time.time()
    objs = []
    procs = []
    for src in ("sho_plan.cpp", "sho_setup.cpp"):
        o = os.path.join(bdir, src.rsplit(".", 1)[0] + ".o")
        if sanitize:
            cmd = [CLANGXX] + HOST_FLAGS + SAN + ["-g", "-fno-omit-frame-pointer", "-c",
                                                  os.path.join(CSRC, src), "-o", o]
        else:
            cmd = ["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, src), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(o)
    san_host = [f for x in SAN for f in ("-Xarch_host", x)] if sanitize else []
    for src in ("sho_api.cpp", "sho_server.cpp", "sho_kernels.hip", "sho_kernels_f32.hip"):
        o = os.path.join(bdir, src.rsplit(".", 1)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + HIP_FLAGS + san_host + lang + ["-c", os.path.join(CSRC, src), "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(o)
    bad = [c for c, p in procs if p.wait() != 0]
    if bad:
        raise RuntimeError("compile failed: " + " ".join(bad[0]))
    lib = LIB_ASAN if sanitize else LIB
    tmp = lib + ".tmp"
    link_san = (SAN + ["-shared-libsan"]) if sanitize else []
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + link_san + objs
         + ["-Wl,-rpath,/opt/rocm/lib"], verbose)
    os.replace(tmp, lib)
    if verbose:
        print("built %s in %.1fs" % (lib, time.time() - t0), flush=True)
    return lib


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv)

"""MI355X-native SHO projection library (Baumeister & Tsukamoto, PASC'19).

The compute path is libsho.so (hand-written gfx950 HIP kernels behind a C
ABI, include/sho.h); this package holds its ctypes binding, the autograd
wrapper and the seeded workload generators.  Submodules are imported lazily
so that ``workloads`` can be used without torch or a built library.
"""
import importlib

__all__ = ["binding", "workloads", "autograd", "serve", "Plan", "Graph", "Server",
           "project", "expand", "force"]


def __getattr__(name):
    if name in ("binding", "workloads", "build", "autograd", "serve"):
        return importlib.import_module("." + name, __name__)
    if name in ("Plan", "Graph", "Server", "project", "expand", "force", "load_library",
                "ShoError"):
        return getattr(importlib.import_module(".binding", __name__), name)
    raise AttributeError(name)

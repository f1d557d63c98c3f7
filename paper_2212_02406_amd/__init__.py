"""Nested Neumann (NN) iterative matrix inversion on MI355X (gfx950).

The compute path is the HIP library ``libnn.so`` built from ``csrc/`` and
declared in ``include/nn.h``; ``nn`` is its thin ctypes binding (argument
marshalling only).  ``workloads`` holds the seeded synthetic input
generators.  Submodules are imported on first use so that the input
generators work without a GPU.
"""
import importlib

__all__ = ["nn", "workloads"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)

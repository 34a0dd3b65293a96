"""MI355X space-time multigrid (STMG) for reaction-diffusion problems.

The numerical work runs in libstmg.so (hand-written HIP for gfx950, C ABI in
include/stmg.h); this package is its Python binding.  See `stmg.Handle`.
"""
import importlib

from . import binding  # noqa: F401

__all__ = ["binding", "stmg"]


def __getattr__(name):
    if name in ("stmg", "autograd"):
        return importlib.import_module(__name__ + "." + name)
    raise AttributeError(name)

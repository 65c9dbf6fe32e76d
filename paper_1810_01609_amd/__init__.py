"""MI355X-native Moebius domain-wall fermion propagator solver.

The solver itself is the HIP library ``libmdwf.so`` (C ABI in
``include/mdwf.h``); this package holds its sources (``csrc/``), the build
script, the thin ctypes binding (``mdwf``) and the continuous-batching
serving loop (``serve``).
"""
from . import mdwf  # noqa: F401
from .mdwf import (  # noqa: F401
    Action, CGOpts, Context, MDWFError, F64, F32, F16, BF16, I16, PREC,
)

__all__ = ["mdwf", "Action", "CGOpts", "Context", "MDWFError", "F64", "F32", "F16", "BF16", "I16", "PREC"]

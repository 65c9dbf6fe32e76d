"""CPU oracle for the Moebius domain-wall propagator solve (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The product (the HIP library and its Python binding) never
imports it and shares no code with it.
"""
from .mdwf import *  # noqa: F401,F403
from .mdwf import __all__  # noqa: F401

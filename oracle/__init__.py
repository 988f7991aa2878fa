"""CPU oracle for the MLMC level sampler -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  The GPU library neither imports nor links it, and it imports
nothing from the GPU library.  See oracle.h for what each function follows.
"""
from .oracle import *  # noqa: F401,F403
from .asian_pde import asian_arith_call_pde  # noqa: F401

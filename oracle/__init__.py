"""CPU FP64 oracle for the short-range LJ MD hot path (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  It never imports the HIP package and the HIP package never
imports it.
"""
from .oracle import *  # noqa: F401,F403
from .sph import *  # noqa: F401,F403,E402
from .spme import *  # noqa: F401,F403,E402

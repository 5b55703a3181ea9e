"""CPU FP64 oracle of the sparse FCT hot path (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the HIP library.
"""
from .fct_oracle import *  # noqa: F401,F403
from . import fct_oracle  # noqa: F401
from . import gauss_oracle  # noqa: F401

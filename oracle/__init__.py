"""FP64 CPU oracle for the CLR block product and S^-1/2 (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The library's product path never does.
"""
from .clr_oracle import *  # noqa: F401,F403
from .clr_oracle import __all__  # noqa: F401

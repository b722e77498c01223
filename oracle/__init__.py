"""Plain, slow, FP64 CPU oracle for azimuthal integration.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the test-suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the GPU library.
"""
from .azint_oracle import *  # noqa: F401,F403

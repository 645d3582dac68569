"""FP64 CPU oracle for the Chebyshev density-matrix path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this; only
the tests, the smoke check and the benchmark's CPU-baseline leg may call it.
It shares no code with the HIP path.
"""
from .dm_oracle import *  # noqa: F401,F403
from . import mlp_oracle  # noqa: F401
from . import grid_oracle  # noqa: F401
from . import factored_oracle  # noqa: F401

"""FP64 CPU oracle for band-limited PDE-LDDMM on the state equation (Gauss-Newton).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's CPU
baseline leg may import it; the product library never does, and the two share no code.
"""
from .bl_oracle import *  # noqa: F401,F403
from .bl_oracle import __all__  # noqa: F401

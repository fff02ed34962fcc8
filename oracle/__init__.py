"""FP64 CPU oracle of band-limited PDE-LDDMM: the state-equation method (bl_oracle) and the
deformation-state-equation method (bl_deform), both with Gauss-Newton-Krylov.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's CPU
baseline leg may import it; the product library never does, and the two share no code.
"""
from .bl_oracle import *  # noqa: F401,F403
from .bl_oracle import __all__ as _state_all
from .bl_deform import *  # noqa: F401,F403
from .bl_deform import __all__ as _deform_all

__all__ = list(_state_all) + list(_deform_all)

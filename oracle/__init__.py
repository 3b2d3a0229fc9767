"""FP64 CPU oracle for the D3Q19 MRT permeability solver.

Test infrastructure only: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the library it checks.
"""
from .lbm_oracle import *  # noqa: F401,F403
from .lbm_oracle import __all__  # noqa: F401

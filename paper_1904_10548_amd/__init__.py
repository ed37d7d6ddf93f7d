"""MI355X dual-APG solver for scenario-tree stochastic MPC of drinking-water
networks (Sopasakis et al., arXiv 1904.10548).

The solver is the C-ABI library ``libtapg.so`` (HIP kernels for gfx950 plus
host C++), declared in ``include/tapg.h`` and bound by :mod:`.tapg`.
"""

from . import tapg  # noqa: F401
from .tapg import Solver, TapgError, TAPG_FP32, TAPG_FP64  # noqa: F401

__all__ = ["tapg", "Solver", "TapgError", "TAPG_FP32", "TAPG_FP64"]

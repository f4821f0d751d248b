"""MI355X (gfx950) gradient-guided Monte Carlo SLAM particle update.

The filter runs in the HIP library ``libmcslam.so`` (sources in ``csrc/``,
C ABI in ``include/mcslam.h``); ``abi`` is its ctypes binding with the same
entry-point names.  Paper: T. Nakao et al., "Range-based 6-DoF Monte Carlo
SLAM with Gradient-guided Particle Filter on GPU" (arXiv 2504.18056).
"""

from . import abi  # noqa: F401
from .abi import McsError  # noqa: F401

"""FP64 CPU oracle of the batched MLS-MPM substep (test infrastructure only).

Only the test suite, the smoke check and the bench's CPU-baseline leg import
this package. It shares no code with the HIP library.
"""
from .mpm_oracle import *  # noqa: F401,F403
from . import mpm_oracle  # noqa: F401

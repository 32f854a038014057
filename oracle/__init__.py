"""Plain FP64 CPU oracle for the tetrahedral FMM (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never links or calls it.
"""
from .oracle import *  # noqa: F401,F403

"""FP64 CPU oracle for FMG-FAS-SR (test infrastructure only).

Only ``tests/``, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  The HIP product path never does.
"""
from .oracle import *  # noqa: F401,F403

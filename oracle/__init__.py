"""Plain FP64 CPU oracle for the short-range MD path (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product path never does, and nothing here imports
the product package except its seeded input generators.
"""
from .oracle import *  # noqa: F401,F403

"""Plain FP64 CPU oracle for the Hermite wave-equation half step.

Test infrastructure only: the test-suite, the smoke check and the benchmark's
CPU-baseline leg import this package; the product library never does.
"""
from .oracle import *  # noqa: F401,F403

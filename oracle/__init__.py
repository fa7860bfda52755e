"""FP64 CPU oracle for structured random phase retrieval (test infrastructure only).

Imported by the test-suite, the smoke check and the benchmark's CPU-baseline leg;
never by the library or its binding.
"""
from .sr_oracle import *  # noqa: F401,F403
from . import sr_oracle  # noqa: F401

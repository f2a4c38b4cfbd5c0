"""FP64 CPU oracle for the ImaSk hot path (arXiv 2412.10249).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  The numerics
live in ``imask_oracle.c`` (plain C, double precision, OpenMP over rays and
angles); this module is the ctypes shim plus numpy conveniences, and
``steps.py`` holds the step-size theory (Sec. 3.5-3.6).

Parity status of each function is listed in the module docstrings of the
tests that pin it (``tests/test_oracle_*.py``).
"""
from .core import *  # noqa: F401,F403
from . import steps  # noqa: F401

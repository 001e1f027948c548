"""CPU oracle for the Giada-Marsili likelihood GA (test infrastructure only).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product path (the HIP library and its binding)
never does. See oracle.c for what each routine computes and which passage of
the paper it follows.
"""
from .oracle import *  # noqa: F401,F403

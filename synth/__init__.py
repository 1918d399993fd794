"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the preconditioner: only grids, seeded
fields, source positions and nodal source samples.  Both the oracle and the
HIP path consume what it produces; neither is imported from here.
"""
from .problems import *  # noqa: F401,F403

"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

Input generation only: finite-element / finite-difference pencils, random
coefficient fields, target windows and circular contours.  Nothing here
performs any step of the contour-integral eigensolver.
"""
from . import pencils, configs  # noqa: F401

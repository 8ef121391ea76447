"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke check.

This package holds plain data only (physical constants, grid sizes, sample
counts, seeds) and a few neutral field generators for the test states.  It
does none of the method's arithmetic: no equation of state, no flux, no
sampling of bubble clouds.  Both the library and the oracle take their inputs
from here.
"""
from .configs import *  # noqa: F401,F403

"""Seeded synthetic workloads shared by the oracle checks, the GPU tests and the bench.

This package generates inputs only (floorplans, variation fields, power traces). It holds
none of the thermal method's arithmetic, and imports neither ``oracle`` nor the GPU package.
"""
from .gen import *  # noqa: F401,F403

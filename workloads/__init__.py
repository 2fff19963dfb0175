"""Seeded synthetic inputs shared by the HIP path, the CPU oracle, tests and benchmarks.

This package only draws input data: velocity models, source and receiver positions,
shot sizes and arrival times.  It holds none of the finite-difference method's
arithmetic (no time step, no wavelet, no sponge, no stencil); each side computes
those in its own code from the data produced here.
"""
from .synthetic import *  # noqa: F401,F403

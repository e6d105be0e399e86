"""Stochastic multiscale flux basis for coupled Stokes-Darcy flow on MI355X.

The compute path is libsdmm.so (hand-written HIP for gfx950, C ABI declared
in include/sdmm.h); ``paper_1802_06263_amd.sdmm`` is its ctypes binding.
"""
from . import sdmm  # noqa: F401
from .sdmm import Context, SdmmError, load  # noqa: F401

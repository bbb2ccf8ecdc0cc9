"""Seeded synthetic inputs shaped like the paper's workloads.

Used by both the oracle-side tests and the GPU path; holds no arithmetic of the
method itself (the low-rank construction uses scipy's FFT/DCT routines, which
neither the oracle nor the HIP library uses).
"""
from .synth import *  # noqa: F401,F403

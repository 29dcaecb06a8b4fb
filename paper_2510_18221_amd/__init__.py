"""MI355X (gfx950) world step of the large-population ecological simulator of
arXiv 2510.18221: per-agent-policy forward, sampling, conflict resolution,
regrowth, births and deaths with Gaussian mutation, as HIP kernels behind the
C ABI of include/eco.h.  `eco.World` is the Python binding.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "eco"]

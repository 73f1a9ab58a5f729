"""MI355X (gfx950) two-component pseudopotential lattice Boltzmann hot path.

Implements the per-time-step method of Chen et al., "Improvement of
Solid-Fluid Interaction Scheme in Lattice Boltzmann Immiscible Pseudopotential
Models" (arXiv 2505.22256) as hand-written HIP kernels behind the C ABI in
include/lbm.h.  ``lbm`` is the Python binding, ``workloads`` the seeded input
generators, ``build`` the in-tree hipcc build.
"""
from . import workloads  # noqa: F401

__all__ = ["lbm", "workloads", "build"]

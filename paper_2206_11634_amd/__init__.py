"""MI355X-native sharp-interface metaball-DEM / lattice Boltzmann hot path.

The compute path lives in the HIP shared library built from ``csrc/`` and is
reached through :mod:`paper_2206_11634_amd.binding` (a ctypes layer over the
C-ABI declared in ``include/mdlbm.h``).  Importing this package loads nothing;
``binding.load()`` raises if the library has not been built.
"""

__all__ = ["binding", "workloads"]

"""MI355X (gfx950) nodal DG discrete-Boltzmann BGK solver.

The solver itself is the HIP library ``libdgbgk.so`` (C ABI in
``include/dgbgk.h``); this package holds its sources (``csrc/``), the build
step (``build.py``) and the ctypes binding (``binding.py``).
"""
from .binding import (BC_DIFFUSE_WALL, BC_PERIODIC, Batch, DgbgkError, Server, Solver, lib, required_bytes,
                      tau_from_kn, velocity_set, velset_gh, velset_nc, version)

__all__ = ["Solver", "Batch", "Server", "DgbgkError", "lib", "velset_gh", "velset_nc", "velocity_set",
           "tau_from_kn", "required_bytes", "version", "BC_PERIODIC", "BC_DIFFUSE_WALL"]

"""libpdbm: gfx950 (MI355X) implementation of the per-timestep update of the
polar-coordinate lattice Boltzmann kinetic model of detonation (Lin, Xu,
Zhang, Li, arXiv:1308.0653).

The compute path is the HIP library ``libpdbm.so`` (C ABI in include/pdbm.h);
``paper_1308_0653_amd.pdbm`` is its ctypes binding and
``paper_1308_0653_amd.workloads`` describes the seeded synthetic inputs.
Importing the package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["pdbm", "workloads", "build"]

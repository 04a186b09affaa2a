"""MI355X-native coupled lattice-Boltzmann / multiparticle-collision time step.

The compute path is the HIP library ``liblbmpcd.so`` built from ``csrc/``; the
Python binding in :mod:`paper_2004_00304_amd.lbmpcd` marshals arguments to its
C ABI and nothing else.  Importing this package does not load the library;
importing :mod:`paper_2004_00304_amd.lbmpcd` does, and fails loudly when it has
not been built.
"""

__all__ = ["workloads"]

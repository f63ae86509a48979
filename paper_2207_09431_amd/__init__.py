"""MI355X-native phase-field power-law lattice Boltzmann step (arXiv 2207.09431).

Submodules:
  pflbm   -- binding of the HIP library libpflbm.so (C ABI in include/pflbm.h)
  inputs  -- seeded synthetic inputs (bubble fields, noise, workload presets)
  build   -- hipcc build of the library
Importing the package loads nothing; the library is opened on first use.
"""
__all__ = ["pflbm", "inputs", "build"]

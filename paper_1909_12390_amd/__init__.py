"""MI355X-native multi-component pseudo-potential lattice Boltzmann step.

The compute path lives in the HIP/C++ shared library built from ``csrc/`` and
declared in ``include/lbm.h``; ``lbm`` is its ctypes binding (argument
marshalling only).  Importing this package loads nothing; the library is loaded
on first use and its absence is an error.
"""
__all__ = ["inputs", "lbm"]

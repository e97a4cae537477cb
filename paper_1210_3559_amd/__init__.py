"""MI355X-native Sutton-Chen molecular dynamics for free nickel clusters.

The compute path is the C-ABI library ``libscmd.so`` (HIP kernels for gfx950,
declared in ``include/scmd.h``); ``paper_1210_3559_amd.scmd`` is its thin
ctypes binding and ``paper_1210_3559_amd.inputs`` the seeded input
generators.  Importing this package loads nothing; the binding loads the
library on first use and raises if it has not been built.
"""
__all__ = ["scmd", "inputs"]

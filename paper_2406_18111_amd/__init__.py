"""MI355X-native FindRepeats (Yadav et al., ASPLOS'25, Section 4.2, Algorithm 2).

The analysis runs in the HIP library libapo.so (C ABI in include/apo.h);
this package holds its build script, the ctypes binding and the synthetic
input generators.  Importing the package does not load the library; use
:func:`paper_2406_18111_amd.load` or :class:`paper_2406_18111_amd.Context`.
"""
from ._lib import (APO_MAX_N, COUNTERS, OCC_DTYPE, ROW_DTYPE, STAGES, ApoError, Context, load)  # noqa: F401

__all__ = ["Context", "ApoError", "load", "ROW_DTYPE", "OCC_DTYPE", "STAGES", "COUNTERS", "APO_MAX_N"]

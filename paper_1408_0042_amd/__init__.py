"""MI355X-native block PLHR eigensolver (HIP for gfx950 behind a C ABI).

See include/plhr.h for the C interface; ``paper_1408_0042_amd.plhr.Solver``
is the Python binding (argument marshalling only).
"""
from . import _lib  # noqa: F401

__all__ = ["_lib"]

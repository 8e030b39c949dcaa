"""MI355X (gfx950) hot path of the Eulerian solvent-excluded surface method.

The computation lives in the HIP library built from csrc/ (C-ABI in
include/eses.h); `eses` is its Python binding.
"""
from . import eses  # noqa: F401

__all__ = ["eses"]

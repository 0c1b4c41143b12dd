"""MI355X-native RMTR hot path for pressure-induced phase-field fracture.

The product is the HIP library librmtr.so (C-ABI in include/rmtr.h); the
`binding` module is its thin Python front end.
"""
from . import binding
from .binding import Context, default_params, load

__all__ = ["binding", "Context", "default_params", "load"]

"""Exact analytic SASA and Cartesian derivatives on MI355X (gfx950).

The HIP library ``libsasa_hip.so`` does all the work; this package only
marshals arguments (``_lib``), wraps a context (``SasaContext``), exposes a
``torch.autograd.Function`` (``sasa_autograd``) and a continuous-batching
server (``server``).
"""
from . import _lib
from ._lib import SasaError
from .context import SasaContext

__all__ = ["SasaContext", "SasaError", "_lib"]

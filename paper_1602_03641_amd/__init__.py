"""MI355X-native hybrid-dimensional VAG Darcy flow + upwind transport.

The compute path is ``libvag.so`` (HIP kernels for gfx950 behind the C-ABI of
``include/vag.h``); ``vag`` is its Python binding.
"""
from . import vag  # noqa: F401

__all__ = ["vag"]

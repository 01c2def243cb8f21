"""MI355X non-singular boundary-integral / Fourier space-time solver.

The computation lives in ``libbem.so`` (HIP kernels for gfx950, C ABI in
``include/bem.h``); this package only marshals arguments (``native``) and
keeps the device buffers of a surface together (``surface``).
"""
from . import native  # noqa: F401
from .surface import DeviceQuadSurface, DeviceSurface, host_surface  # noqa: F401

"""MI355X-native Image Source Method (room impulse responses) with HIP kernels for gfx950.

The library is ``libism.so`` (C ABI in include/ism.h); ``ism`` is its ctypes binding.
"""
from . import ism  # noqa: F401
from .ism import Room, Simulator, simulate  # noqa: F401

"""GOSMA branch-and-bound bound evaluation on MI355X (gfx950).

The HIP library (csrc/, built into libgosma.so) holds every step of the hot
path; gosma.py is its ctypes binding.
"""
from .gosma import Context, GosmaError, lib  # noqa: F401
